"""Pins of the CPU oracle against definitions, closed forms and invariants.

Nothing here compares the oracle with itself: each check sets an oracle
routine against an independently built object (kron-built Jordan-Wigner
matrices, the dense Fock Hamiltonian of eq. 1 built from v_pqrs, a closed
form derived from the operator algebra, or a textbook dense algorithm).
"""
import numpy as np
import pytest

import synth
from oracle import fermion as F
from oracle import hamiltonian as OH
from oracle import hf as HF
from oracle import lanczos as OL
from oracle import mps as M
from oracle import thc as TH


def _normalised_random_mps(rng, n, D):
    psi = synth.random_mps_tensors(rng, n, D)
    return M.scale(psi, 1.0 / M.norm(psi))


def _dense(m):
    return m.toarray() if hasattr(m, "toarray") else m


# --------------------------------------------------------------------------
# Jordan-Wigner algebra (Sec. 3.1 JW substitution, App. C)
# --------------------------------------------------------------------------

def test_car_relations():
    n = 6
    a = [_dense(x) for x in F.annihilators(n)]
    I = np.eye(2 ** n)
    for i in range(n):
        for j in range(n):
            anti = a[i] @ a[j].T + a[j].T @ a[i]
            assert np.array_equal(anti, I if i == j else 0 * I)
            assert np.array_equal(a[i] @ a[j] + a[j] @ a[i], 0 * I)


def test_app_c_local_operators():
    # b_up = c (x) I2, b_down = Z (x) c on one spatial orbital (App. C)
    a0 = _dense(F.jw_annihilator(0, 2))
    a1 = _dense(F.jw_annihilator(1, 2))
    assert np.array_equal(a0, np.kron(F.C, F.I2))
    assert np.array_equal(a1, np.kron(F.Z, F.C))
    # c annihilates an occupied orbital: c|1> = |0>
    assert F.C[0, 1] == 1.0 and F.C.sum() == 1.0


def test_dense_vector_ops_match_matrices():
    n = 6
    rng = np.random.default_rng(1)
    vec = rng.standard_normal(2 ** n)
    for j in range(n):
        a = _dense(F.jw_annihilator(j, n))
        assert np.allclose(F.apply_a(vec, j, n), a @ vec, atol=0, rtol=0)
        assert np.allclose(F.apply_a(vec, j, n, dag=True), a.T @ vec, atol=0, rtol=0)


# --------------------------------------------------------------------------
# Elementary MPO (eq. elementary_MPO): contracting the W's gives sum_j y_j a_j
# --------------------------------------------------------------------------

@pytest.mark.parametrize("dag", [False, True])
def test_layer_mpo_contracts_to_one_body_operator(dag):
    n = 6
    rng = np.random.default_rng(2)
    y = rng.standard_normal(n)
    ref = sum(y[j] * _dense(F.jw_annihilator(j, n)) for j in range(n))
    if dag:
        ref = ref.T
    got = M.mpo_to_dense(M.layer_mpo(y, dag))
    assert np.max(np.abs(got - ref)) < 1e-14


@pytest.mark.parametrize("dag", [False, True])
def test_apply_layer_on_mps(dag):
    n = 8
    rng = np.random.default_rng(3)
    psi = _normalised_random_mps(rng, n, 8)
    y = rng.standard_normal(n)
    op = sum(y[j] * _dense(F.jw_annihilator(j, n)) for j in range(n))
    if dag:
        op = op.T
    got = M.to_dense(M.apply_layer(psi, y, dag))
    assert np.max(np.abs(got - op @ M.to_dense(psi))) < 1e-13
    assert M.bonds(M.apply_layer(psi, y, dag))[1:-1] == [2 * b for b in M.bonds(psi)[1:-1]]


# --------------------------------------------------------------------------
# THC-MPO reproduces eq. (1); kinetic split is exact (App. D)
# --------------------------------------------------------------------------

def _factors(L, N, seed=0):
    rng = np.random.default_rng(seed)
    return synth.thc_factors(rng, L, N)


def test_one_particle_sector_closed_form():
    # one electron of spin up: <p|H|k> = t_pk + 1/2 sum_r v_prrk (operator order of eq. 1)
    L, N = 3, 4
    t, chi, zeta = _factors(L, N, seed=5)
    v = TH.thc_v(chi, zeta)
    H = _dense(F.hamiltonian_sparse(t, v))
    n = 2 * L
    idx = [1 << (n - 1 - 2 * p) for p in range(L)]  # single up electron in orbital p
    sub = H[np.ix_(idx, idx)]
    ref = t + 0.5 * np.einsum("prrk->pk", v)
    assert np.max(np.abs(sub - ref)) < 1e-13


def test_thc_mpo_products_equal_eq1():
    L, N = 3, 4
    t, chi, zeta = _factors(L, N)
    v = TH.thc_v(chi, zeta)
    Hv = _dense(F.hamiltonian_sparse(0 * t, v))
    n = 2 * L
    acc = np.zeros((2 ** n, 2 ** n))
    for nu, sp_, mu, s in TH.v_terms(N):
        ops = [
            M.mpo_to_dense(M.layer_mpo(TH.spin_site_coeffs(chi[:, mu], s), True)),
            M.mpo_to_dense(M.layer_mpo(TH.spin_site_coeffs(chi[:, mu], s), False)),
            M.mpo_to_dense(M.layer_mpo(TH.spin_site_coeffs(chi[:, nu], sp_), True)),
            M.mpo_to_dense(M.layer_mpo(TH.spin_site_coeffs(chi[:, nu], sp_), False)),
        ]
        acc += 0.5 * zeta[mu, nu] * (ops[0] @ ops[1] @ ops[2] @ ops[3])
    assert np.max(np.abs(acc - Hv)) < 1e-13 * max(1.0, np.max(np.abs(Hv)))


def test_kinetic_split_exact():
    L = 4
    t, _, _ = _factors(L, 2)
    T = _dense(F.hamiltonian_sparse(t, np.zeros((L,) * 4)))
    lam, u = TH.kinetic_split(t)
    n = 2 * L
    acc = np.zeros_like(T)
    for i in range(L):
        for s in (0, 1):
            cre = M.mpo_to_dense(M.layer_mpo(TH.spin_site_coeffs(u[:, i], s), True))
            ann = M.mpo_to_dense(M.layer_mpo(TH.spin_site_coeffs(u[:, i], s), False))
            acc += lam[i] * cre @ ann
    assert np.max(np.abs(acc - T)) < 1e-13


def test_dense_vector_H_matches_matrix():
    L, N = 4, 8
    t, chi, zeta = _factors(L, N)
    v = TH.thc_v(chi, zeta)
    H = F.hamiltonian_sparse(t, v)
    vec = np.random.default_rng(4).standard_normal(2 ** (2 * L))
    assert np.max(np.abs(F.apply_H_dense(vec, t, v) - H @ vec)) < 1e-12 * np.max(np.abs(H @ vec))


# --------------------------------------------------------------------------
# Hartree-Fock energy: closed form vs dense eq. (1)
# --------------------------------------------------------------------------

def test_hf_closed_form_vs_dense():
    L, N = 4, 8
    t, chi, zeta = _factors(L, N, seed=7)
    v = TH.thc_v(chi, zeta)
    H = F.hamiltonian_sparse(t, v)
    n = 2 * L
    for n_elec in (2, 4, 6):
        occ = synth.hartree_fock_occupation(L, n_elec)
        idx = sum(o << (n - 1 - j) for j, o in enumerate(occ))
        e_dense = H[idx, idx]
        e_cf = HF.closed_shell_energy(t, v, range(n_elec // 2))
        e_det = HF.determinant_energy(t, v, occ)
        assert abs(e_dense - e_cf) < 1e-12 * max(1, abs(e_dense))
        assert abs(e_dense - e_det) < 1e-12 * max(1, abs(e_dense))
    # an open-shell determinant (one up electron in 0, one down in 2)
    occ = [1, 0, 0, 0, 0, 1, 0, 0]
    idx = sum(o << (n - 1 - j) for j, o in enumerate(occ))
    assert abs(H[idx, idx] - HF.determinant_energy(t, v, occ)) < 1e-12 * max(1, abs(H[idx, idx]))


def test_hf_energy_via_mps_path():
    # <HF| H |HF> with the compressed THC-MPO path equals the closed form
    L, N = 4, 8
    t, chi, zeta = _factors(L, N, seed=8)
    v = TH.thc_v(chi, zeta)
    occ = synth.hartree_fock_occupation(L, 4)
    hf = synth.occupation_mps_tensors(occ)
    Hhf = OH.apply_H(hf, t, chi, zeta, D=16)
    e = M.overlap(hf, Hhf)
    assert abs(e - HF.closed_shell_energy(t, v, [0, 1])) < 1e-12 * max(1, abs(e))


# --------------------------------------------------------------------------
# Compression (Fig. 3): exactness, idempotence, canonical form, Eckart-Young
# --------------------------------------------------------------------------

def test_compress_exact_when_untruncated():
    rng = np.random.default_rng(9)
    psi = _normalised_random_mps(rng, 8, 16)
    c = M.compress(psi, 16)
    assert np.max(np.abs(M.to_dense(c) - M.to_dense(psi))) < 1e-13
    assert M.left_canonical_error(c) < 1e-13


def test_right_canonical_form_checker():
    # the QR sweep gives orthonormal rows at sites 1..n-1 and the same state;
    # a generic random MPS is far from that form
    rng = np.random.default_rng(12)
    psi = _normalised_random_mps(rng, 8, 8)
    rc = M.right_canonicalize(psi)
    assert M.right_canonical_error(rc) < 1e-13
    assert M.right_canonical_error(psi) > 1e-2
    assert np.max(np.abs(M.to_dense(rc) - M.to_dense(psi))) < 1e-13
    # the norm sits on site 0
    a0 = rc[0].reshape(-1)
    assert abs(np.linalg.norm(a0) - M.norm(psi)) < 1e-13


def test_compress_discarded_weight_and_idempotence():
    rng = np.random.default_rng(10)
    n = 10
    psi = _normalised_random_mps(rng, n, 32)
    D = 8
    rec = []
    c = M.compress(psi, D, record=rec)
    disc = sum(float(np.sum(s[D:] ** 2)) for s in rec)
    err = np.linalg.norm(M.to_dense(c) - M.to_dense(psi)) ** 2
    # successive truncation errors are orthogonal (left -> right sweep)
    assert abs(err - disc) < 1e-12
    # first bond: Eckart-Young against the dense SVD of the state
    dense = M.to_dense(psi).reshape(2, -1)
    s_dense = np.linalg.svd(dense, compute_uv=False)
    assert np.allclose(rec[0], s_dense[: rec[0].size], atol=1e-13)
    c2 = M.compress(c, D)
    assert np.max(np.abs(M.to_dense(c2) - M.to_dense(c))) < 1e-13
    assert M.left_canonical_error(c) < 1e-12
    assert max(M.bonds(c)) <= D


def test_compress_zero_state_keeps_bond_one():
    rng = np.random.default_rng(11)
    psi = M.scale(_normalised_random_mps(rng, 6, 4), 0.0)
    c = M.compress(psi, 4)
    assert max(M.bonds(c)) == 1
    assert np.all(M.to_dense(c) == 0)


def test_direct_sum_and_overlap():
    rng = np.random.default_rng(12)
    a = _normalised_random_mps(rng, 8, 8)
    b = _normalised_random_mps(rng, 8, 4)
    s = M.direct_sum([(0.3, a), (-1.7, b)])
    ref = 0.3 * M.to_dense(a) - 1.7 * M.to_dense(b)
    assert np.max(np.abs(M.to_dense(s) - ref)) < 1e-14
    assert abs(M.overlap(a, b) - M.to_dense(a) @ M.to_dense(b)) < 1e-14


# --------------------------------------------------------------------------
# H|psi> untruncated: MPS path == dense eq. (1); both sum orders; hermiticity
# --------------------------------------------------------------------------

@pytest.fixture(scope="module")
def small_case():
    t, chi, zeta, sites = synth.make_workload("L4_N8_D16")
    psi = M.scale(sites, 1.0 / M.norm(sites))
    v = TH.thc_v(chi, zeta)
    return t, chi, zeta, v, psi


def test_apply_H_untruncated_matches_dense(small_case):
    t, chi, zeta, v, psi = small_case
    ref = F.apply_H_dense(M.to_dense(psi), t, v)
    for mode in ("tree", "sequential"):
        out = OH.apply_H(psi, t, chi, zeta, D=16, mode=mode)
        got = M.to_dense(out)
        assert np.linalg.norm(got - ref) < 1e-12 * np.linalg.norm(ref), mode


def test_hermiticity(small_case):
    t, chi, zeta, v, psi = small_case
    rng = np.random.default_rng(13)
    phi = _normalised_random_mps(rng, 8, 16)
    a = M.overlap(phi, OH.apply_H(psi, t, chi, zeta, 16))
    b = M.overlap(OH.apply_H(phi, t, chi, zeta, 16), psi)
    assert abs(a - b) < 1e-12 * max(abs(a), 1.0)


def test_particle_number_and_sz_conserved():
    L, N = 4, 8
    t, chi, zeta = _factors(L, N, seed=14)
    occ = [1, 0, 0, 1, 1, 1, 0, 0]  # N = 4, 2Sz = 0
    psi = synth.occupation_mps_tensors(occ)
    out = M.to_dense(OH.apply_H(psi, t, chi, zeta, 16))
    nn = F.number_operator_dense(8)
    sz = F.sz_dense(8)
    w = out ** 2 / np.sum(out ** 2)
    assert abs(w @ nn - 4) < 1e-12 and w @ (nn - 4) ** 2 < 1e-12
    assert abs(w @ sz) < 1e-12 and w @ sz ** 2 < 1e-12


def test_sum_compress_untruncated_linear():
    rng = np.random.default_rng(15)
    terms = [_normalised_random_mps(rng, 6, 2) for _ in range(5)]
    coeffs = [0.5, -1.0, 2.0, 0.25, -0.75]
    out = OH.sum_compress(coeffs, terms, D=8)
    ref = sum(c * M.to_dense(m) for c, m in zip(coeffs, terms))
    assert np.linalg.norm(M.to_dense(out) - ref) < 1e-13 * np.linalg.norm(ref)


# --------------------------------------------------------------------------
# Lanczos: untruncated MPS Lanczos == textbook dense Lanczos
# --------------------------------------------------------------------------

def test_mps_lanczos_matches_dense_lanczos():
    L, N = 3, 4
    t, chi, zeta = _factors(L, N, seed=16)
    v = TH.thc_v(chi, zeta)
    occ = synth.hartree_fock_occupation(L, 2)
    hf = synth.occupation_mps_tensors(occ)
    K = 6
    st = OL.KrylovState(hf, K)
    ritz_mps = []
    for _ in range(K):
        rg, rt, b = OL.krylov_step(st, t, chi, zeta, D=8)
        ritz_mps.append(rg)
    H = F.hamiltonian_sparse(t, v)
    dense = OL.dense_lanczos(lambda x: H @ x, M.to_dense(hf), K)
    for a, b in zip(ritz_mps, dense):
        assert np.allclose(a, b, atol=1e-10, rtol=0)
    # the Krylov space grows to the full sector here; ground energy of the
    # (N=2, Sz=0) sector is reached by Lanczos
    nn = F.number_operator_dense(6)
    sz = F.sz_dense(6)
    sec = np.where((nn == 2) & (sz == 0))[0]
    e0 = np.linalg.eigvalsh(H.toarray()[np.ix_(sec, sec)])[0]
    assert abs(ritz_mps[-1][0] - e0) < 1e-8


def test_two_trees_order_is_exact_untruncated():
    # the two-part summation order (reading R13) changes only the order of the
    # compressed additions: untruncated it is eq. (1) applied densely
    rng = np.random.default_rng(31)
    L, N = 3, 4
    t, chi, zeta = synth.thc_factors(rng, L, N)
    psi = synth.random_mps_tensors(rng, 2 * L, 8)
    got = M.to_dense(OH.apply_H(psi, t, chi, zeta, 8, mode="two_trees"))
    want = F.apply_H_dense(M.to_dense(psi), t, TH.thc_v(chi, zeta))
    assert np.linalg.norm(got - want) < 1e-12 * np.linalg.norm(want)
    # with every V term in the first half the order falls back to the single tree
    z1 = zeta.copy()
    z1[:, N // 2:] = 0.0
    a = M.to_dense(OH.apply_H(psi, t, chi, z1, 4, mode="two_trees"))
    b = M.to_dense(OH.apply_H(psi, t, chi, z1, 4, mode="tree"))
    assert np.array_equal(a, b)
