"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Tolerances (FP64 path): untruncated results 1e-12 relative to the dense
reference; truncated results compare mode-matched (same tree order) to the
oracle's compressed state at 1e-9 relative, where the gap at the cut is
reported (a near-degenerate cut makes the truncation ill-conditioned).
"""
import numpy as np
import pytest

import synth
from oracle import fermion as F
from oracle import hamiltonian as OH
from oracle import lanczos as OL
from oracle import mps as M
from oracle import thc as TH

pytestmark = pytest.mark.gpu

# The SVD methods of the truncation step: 0 = eigenpairs of the Gram matrix
# (default; two-stage tridiagonalisation; jobs whose kept eigenvalues reach
# the Gram route's noise floor, 32 m eps of the largest, get a second Gram
# level), 8 = the same with the one-stage tridiagonalisation, 1 = one-sided
# block Jacobi for every job.  All meet the untruncated FP64 bar of 1e-12 on
# the Hartree-Fock-derived states used here (rank-deficient, Schmidt spectra
# spanning > 20 decades).
SVD_MODES = [(0, 1e-12), (8, 1e-12), (1, 1e-12)]


def _norm_mps(rng, n, D):
    psi = synth.random_mps_tensors(rng, n, D)
    return M.scale(psi, 1.0 / M.norm(psi))


@pytest.fixture(scope="module")
def thck():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2409_12708_amd as p
    return p


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def test_overlap_matches_oracle(thck):
    rng = np.random.default_rng(1)
    a = _norm_mps(rng, 10, 16)
    b = _norm_mps(rng, 10, 8)
    t, chi, zeta = synth.thc_factors(np.random.default_rng(0), 5, 2)
    ctx = thck.Context(t, chi, zeta)
    da, db = thck.DeviceMPS.from_sites(a), thck.DeviceMPS.from_sites(b)
    got = ctx.overlap(da, db)
    ref = M.to_dense(a) @ M.to_dense(b)
    assert abs(got - ref) < 1e-13 * max(1, abs(ref)), (got, ref)
    assert abs(ctx.overlap(da, da) - 1.0) < 1e-13


@pytest.mark.parametrize("dag", [0, 1])
@pytest.mark.parametrize("D", [16, 4])
def test_layer_compress(thck, dag, D):
    rng = np.random.default_rng(2 + dag)
    n = 8
    psi = _norm_mps(rng, n, 16)
    y = rng.standard_normal(n)
    t, chi, zeta = synth.thc_factors(np.random.default_rng(0), n // 2, 2)
    ctx = thck.Context(t, chi, zeta)
    st = thck.ThcStats()
    out = ctx.apply_layer(thck.DeviceMPS.from_sites(psi), y, dag, D, stats=st)
    got = M.to_dense(out.to_sites())
    ref_state = M.compress(M.apply_layer(psi, y, bool(dag)), D)
    ref = M.to_dense(ref_state)
    tol = 1e-12 if D >= 16 else 1e-9
    assert _rel(got, ref) < tol, (_rel(got, ref), st.as_dict())
    assert out.bond_list() == M.bonds(ref_state)


@pytest.mark.parametrize("flags,tol", SVD_MODES)
def test_compress_hf_rank_deficient(thck, flags, tol):
    # bond-1 product state: every layer output is rank deficient in the padding
    L = 4
    occ = synth.hartree_fock_occupation(L, 4)
    hf = synth.occupation_mps_tensors(occ)
    rng = np.random.default_rng(5)
    y = rng.standard_normal(2 * L)
    t, chi, zeta = synth.thc_factors(np.random.default_rng(0), L, 2)
    ctx = thck.Context(t, chi, zeta)
    out = ctx.apply_layer(thck.DeviceMPS.from_sites(hf), y, 0, 8, flags=flags)
    ref_state = M.compress(M.apply_layer(hf, y, False), 8)
    assert _rel(M.to_dense(out.to_sites()), M.to_dense(ref_state)) < tol
    assert out.bond_list() == M.bonds(ref_state)


@pytest.mark.parametrize("k", [1, 2, 3, 5])
def test_sum_compress_untruncated(thck, k):
    rng = np.random.default_rng(10 + k)
    n = 8
    terms = [_norm_mps(rng, n, 2) for _ in range(k)]
    coeffs = list(rng.standard_normal(k))
    t, chi, zeta = synth.thc_factors(np.random.default_rng(0), n // 2, 2)
    ctx = thck.Context(t, chi, zeta)
    out = ctx.sum_compress(coeffs, [thck.DeviceMPS.from_sites(x) for x in terms], D=16)
    ref = sum(c * M.to_dense(x) for c, x in zip(coeffs, terms))
    assert _rel(M.to_dense(out.to_sites()), ref) < 1e-12
    # the output is right-canonical (sites 1..n-1 have orthonormal rows) and says so
    assert M.right_canonical_error(out.to_sites()) < 1e-12
    assert out.canonical


def test_sum_compress_truncated_tree_order(thck):
    rng = np.random.default_rng(20)
    n = 10
    terms = [_norm_mps(rng, n, 8) for _ in range(7)]
    coeffs = list(rng.standard_normal(7))
    t, chi, zeta = synth.thc_factors(np.random.default_rng(0), n // 2, 2)
    ctx = thck.Context(t, chi, zeta)
    out = ctx.sum_compress(coeffs, [thck.DeviceMPS.from_sites(x) for x in terms], D=8)
    ref = M.to_dense(OH.sum_compress(coeffs, terms, D=8))
    assert _rel(M.to_dense(out.to_sites()), ref) < 1e-9


def test_apply_H_small_dense(thck):
    # L=4 (8 sites), N=8, D=16: exact, against the dense Fock H of eq. (1)
    t, chi, zeta, sites = synth.make_workload("L4_N8_D16")
    psi = M.scale(sites, 1.0 / M.norm(sites))
    ctx = thck.Context(t, chi, zeta)
    st = thck.ThcStats()
    out = ctx.apply_H(thck.DeviceMPS.from_sites(psi), D=16, stats=st)
    got = M.to_dense(out.to_sites())
    ref = F.apply_H_dense(M.to_dense(psi), t, TH.thc_v(chi, zeta))
    err = _rel(got, ref)
    print(f"L4 N8 D16: rel err {err:.3e}, stats {st.as_dict()}")
    assert err < 1e-12
    assert st.n_compressions == 2 * 2 * 8 + 2 * 4 * 64 + 2 * 8 + (4 * 64 + 8 - 1)


def test_apply_H_truncated_matches_oracle_tree(thck):
    # truncated (D=8 < Schmidt rank 16): mode-matched against the oracle's tree sum
    L, N = 4, 6
    rng = np.random.default_rng(30)
    t, chi, zeta = synth.thc_factors(rng, L, N)
    psi = _norm_mps(rng, 2 * L, 16)
    ctx = thck.Context(t, chi, zeta)
    out = ctx.apply_H(thck.DeviceMPS.from_sites(psi), D=8)
    ref = M.to_dense(OH.apply_H(psi, t, chi, zeta, D=8, mode="tree"))
    err = _rel(M.to_dense(out.to_sites()), ref)
    print(f"truncated L4 N6 D8: rel err vs oracle tree {err:.3e}")
    assert err < 1e-8


@pytest.mark.parametrize("flags,tol", SVD_MODES)
def test_hf_energy_gpu(thck, flags, tol):
    L, N = 4, 8
    t, chi, zeta = synth.thc_factors(np.random.default_rng(8), L, N)
    v = TH.thc_v(chi, zeta)
    from oracle import hf as HF
    occ = synth.hartree_fock_occupation(L, 4)
    hf = synth.occupation_mps_tensors(occ)
    ctx = thck.Context(t, chi, zeta)
    dhf = thck.DeviceMPS.from_sites(hf)
    e = ctx.overlap(dhf, ctx.apply_H(dhf, D=16, flags=flags))
    err = abs(e - HF.closed_shell_energy(t, v, [0, 1])) / max(1, abs(e))
    print(f"HF energy flags={flags}: rel err {err:.3e}")
    assert err < tol


@pytest.mark.parametrize("flags,tol", SVD_MODES)
def test_lanczos_small_matches_oracle(thck, flags, tol):
    L, N = 3, 4
    t, chi, zeta = synth.thc_factors(np.random.default_rng(16), L, N)
    occ = synth.hartree_fock_occupation(L, 2)
    hf = synth.occupation_mps_tensors(occ)
    K = 5
    st = OL.KrylovState(hf, K)
    ctx = thck.Context(t, chi, zeta)
    kr = thck.Krylov(ctx, thck.DeviceMPS.from_sites(hf), K, D=8, flags=flags)
    atol = 1e-10
    for i in range(K):
        rg, rt, b = OL.krylov_step(st, t, chi, zeta, D=8)
        g, tt, bb = kr.step()
        print(f"lanczos flags={flags} step {i}: ritz err {np.max(np.abs(g - rg)):.2e}")
        assert np.allclose(g, rg, atol=atol, rtol=0), (i, g, rg)
        assert np.allclose(tt, rt, atol=atol, rtol=0), (i, tt, rt)
        assert abs(bb - b) < atol


def test_apply_H_untruncated_at_tile_size(thck):
    # L=8 (16 sites), N=32, D=256: the largest Schmidt rank of 16 sites is
    # 2^8 = 256, so the compressed result is exact; the interior site matrices
    # have the full 512 x 1024 LQ and 512 x 512 SVD shapes of the L=20 run.
    t, chi, zeta, sites = synth.make_workload("L8_N32_D256")
    psi = M.scale(sites, 1.0 / M.norm(sites))
    ctx = thck.Context(t, chi, zeta)
    st = thck.ThcStats()
    out = ctx.apply_H(thck.DeviceMPS.from_sites(psi), D=256, stats=st)
    got = M.to_dense(out.to_sites())
    ref = F.apply_H_dense(M.to_dense(psi), t, TH.thc_v(chi, zeta))
    err = _rel(got, ref)
    print(f"L8 N32 D256: rel err {err:.3e}, compressions {st.n_compressions}, max bond {st.max_bond}")
    assert err < 1e-12
    assert st.n_compressions == 2 * 2 * 32 + 2 * 4 * 32 * 32 + 2 * 2 * 8 + (4 * 32 * 32 + 2 * 8 - 1)


def test_kernel_timing_flag(thck):
    # THC_FLAG_TIME_KERNELS fills per-kernel device times and flops without
    # changing the result
    t, chi, zeta, sites = synth.make_workload("L4_N8_D16")
    psi = M.scale(sites, 1.0 / M.norm(sites))
    ctx = thck.Context(t, chi, zeta)
    d = thck.DeviceMPS.from_sites(psi)
    s0, s1 = thck.ThcStats(), thck.ThcStats()
    a = M.to_dense(ctx.apply_H(d, D=16, stats=s0).to_sites())
    b = M.to_dense(ctx.apply_H(d, D=16, stats=s1, flags=thck.FLAG_TIME_KERNELS).to_sites())
    assert _rel(b, a) < 1e-14
    k0, k1 = s0.kernels(), s1.kernels()
    assert all(v == (0.0, 0.0, 0, 0.0) for v in k0.values())
    for name in ("lq", "sytrd", "tri_eig", "ormtr", "gemm"):
        ms, fl, n, by = k1[name]
        assert n > 0 and ms > 0.0 and by > 0.0, (name, k1[name])
        if name != "tri_eig":
            assert fl > 0.0
    # the method's bytes of the tridiagonalisation: m^2 + 3m doubles per
    # m x m matrix, against 4m^3/3 flops
    assert k1["sytrd"][3] > 0 and k1["sytrd"][1] > 0
    # one LQ per site of the canonical sweep and one per bond of the SVD sweep
    assert k1["lq"][2] == 2 * k1["sytrd"][2] or k1["lq"][2] > k1["sytrd"][2]


# ---------------------------------------------------------------------------
# Right-canonical inputs: the structured orthogonalisation sweep keeps the
# input's orthonormal rows and factorises only the rest.  The compressed
# state must be the one the plain sweep gives.
# ---------------------------------------------------------------------------

def _rc_mps(rng, n, D):
    return M.right_canonicalize(_norm_mps(rng, n, D))


@pytest.mark.parametrize("dag", [0, 1])
@pytest.mark.parametrize("D", [16, 4])
def test_layer_compress_canonical_input(thck, dag, D):
    rng = np.random.default_rng(40 + dag)
    n = 10
    psi = _rc_mps(rng, n, 16)
    assert M.right_canonical_error(psi) < 1e-13
    y = rng.standard_normal(n)
    t, chi, zeta = synth.thc_factors(np.random.default_rng(0), n // 2, 2)
    ctx = thck.Context(t, chi, zeta)
    ref_state = M.compress(M.apply_layer(psi, y, bool(dag)), D)
    ref = M.to_dense(ref_state)
    tol = 1e-12 if D >= 16 else 1e-9
    outs = {}
    for decl in (False, True):
        out = ctx.apply_layer(thck.DeviceMPS.from_sites(psi, canonical=decl), y, dag, D)
        outs[decl] = out
        err = _rel(M.to_dense(out.to_sites()), ref)
        print(f"layer dag={dag} D={D} declared canonical={decl}: rel err {err:.3e}")
        assert err < tol
        assert out.bond_list() == M.bonds(ref_state)
        assert out.canonical and M.right_canonical_error(out.to_sites()) < 1e-12


@pytest.mark.parametrize("D", [32, 6])
def test_sum_compress_canonical_inputs(thck, D):
    rng = np.random.default_rng(50)
    n = 10
    terms = [_rc_mps(rng, n, 8) for _ in range(3)]
    coeffs = [0.7, -1.3, 0.4]
    t, chi, zeta = synth.thc_factors(np.random.default_rng(0), n // 2, 2)
    ctx = thck.Context(t, chi, zeta)
    ref = M.to_dense(OH.sum_compress(coeffs, terms, D=D))
    for decl in ((False, False, False), (True, True, True), (False, True, False)):
        out = ctx.sum_compress(coeffs, [thck.DeviceMPS.from_sites(x, canonical=c) for x, c in zip(terms, decl)], D=D)
        err = _rel(M.to_dense(out.to_sites()), ref)
        print(f"sum D={D} declared {decl}: rel err {err:.3e}")
        assert err < (1e-12 if D >= 32 else 1e-9)
        assert M.right_canonical_error(out.to_sites()) < 1e-12


# Rank-deficient sums: the Gram route cannot tell a singular value below
# ~sqrt(m eps) s_1 from an exact zero, so every job whose kept eigenvalues
# reach its noise floor goes to Jacobi; both modes meet 1e-12.
@pytest.mark.parametrize("flags,tol", SVD_MODES)
def test_canonical_rank_deficient_product_state(thck, flags, tol):
    # a product state is right-canonical; every layer output and sum in H is
    # rank deficient in its padding, so the rest rows of the structured sweep
    # have exact linear dependencies
    L, N = 4, 8
    t, chi, zeta = synth.thc_factors(np.random.default_rng(8), L, N)
    occ = synth.hartree_fock_occupation(L, 4)
    hf = synth.occupation_mps_tensors(occ)
    ctx = thck.Context(t, chi, zeta)
    ref = F.apply_H_dense(M.to_dense(hf), t, TH.thc_v(chi, zeta))
    for decl in (False, True):
        st = thck.ThcStats()
        out = ctx.apply_H(thck.DeviceMPS.from_sites(hf, canonical=decl), D=16, flags=flags, stats=st)
        err = _rel(M.to_dense(out.to_sites()), ref)
        print(f"H|HF> flags={flags} declared canonical={decl}: rel err {err:.3e}, "
              f"SVD fallbacks {st.svd_fallbacks} of {st.n_compressions * 7} SVDs")
        assert err < tol
        if flags == 0:
            assert st.svd_fallbacks > 0  # the rank-deficient jobs took the Jacobi route
        assert M.right_canonical_error(out.to_sites()) < 1e-12


def test_apply_H_canonical_input_matches_plain(thck):
    # truncated H|psi> (D=8): declared-canonical input against the oracle tree
    L, N = 4, 6
    rng = np.random.default_rng(30)
    t, chi, zeta = synth.thc_factors(rng, L, N)
    psi = M.right_canonicalize(_norm_mps(rng, 2 * L, 16))
    ctx = thck.Context(t, chi, zeta)
    ref = M.to_dense(OH.apply_H(psi, t, chi, zeta, D=8, mode="tree"))
    for decl in (False, True):
        out = ctx.apply_H(thck.DeviceMPS.from_sites(psi, canonical=decl), D=8)
        err = _rel(M.to_dense(out.to_sites()), ref)
        print(f"truncated H|psi> declared canonical={decl}: rel err vs oracle tree {err:.3e}")
        assert err < 1e-8


# ---------------------------------------------------------------------------
# Mixed-precision contractions (thc_prec): the absorb products run in FP32 or
# BF16x3 on MFMA with FP32 accumulation; factorisations, overlaps and the
# Lanczos eigensolve stay FP64.  Untruncated results against the dense FP64
# reference: 1e-5 relative (FP32), 1e-3 (BF16x3).  The error must also sit
# above FP64 rounding, or the reduced-precision path did not run.
# ---------------------------------------------------------------------------
MIXED = [("f32", 1e-5), ("bf16x3", 1e-3)]


@pytest.mark.parametrize("prec,tol", MIXED)
@pytest.mark.parametrize("workload", ["L4_N8_D16", "L8_N32_D256"])
def test_apply_H_mixed_precision_untruncated(thck, prec, tol, workload):
    t, chi, zeta, sites = synth.make_workload(workload)
    psi = M.scale(sites, 1.0 / M.norm(sites))
    ctx = thck.Context(t, chi, zeta)
    D = synth.WORKLOADS[workload]["D"]
    out = ctx.apply_H(thck.DeviceMPS.from_sites(psi), D=D, prec=prec)
    got = M.to_dense(out.to_sites())
    ref = F.apply_H_dense(M.to_dense(psi), t, TH.thc_v(chi, zeta))
    err = _rel(got, ref)
    print(f"{workload} prec={prec}: rel err vs dense FP64 {err:.3e}")
    assert err < tol
    assert err > 1e-13


@pytest.mark.parametrize("prec,tol", MIXED)
def test_lanczos_mixed_precision_energies(thck, prec, tol):
    # Ritz values of a mixed-precision Krylov run against the FP64 oracle
    L, N = 3, 4
    t, chi, zeta = synth.thc_factors(np.random.default_rng(16), L, N)
    occ = synth.hartree_fock_occupation(L, 2)
    hf = synth.occupation_mps_tensors(occ)
    K = 4
    st = OL.KrylovState(hf, K)
    ctx = thck.Context(t, chi, zeta)
    kr = thck.Krylov(ctx, thck.DeviceMPS.from_sites(hf), K, D=8, prec=prec)
    for i in range(K):
        rg, _, _ = OL.krylov_step(st, t, chi, zeta, D=8)
        g, _, _ = kr.step()
        err = np.max(np.abs(g - rg)) / max(1.0, np.max(np.abs(rg)))
        print(f"lanczos prec={prec} step {i}: max Ritz error {err:.2e}")
        assert err < tol
