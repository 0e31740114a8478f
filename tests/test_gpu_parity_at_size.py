"""GPU parity at the throughput shapes and on the configurations that truncate.

* One layer-compression (eq. elementary_MPO applied, then Fig. 3's QR + SVD
  sweeps) and one add-compression (direct sum + compression, Algorithm 1) of
  the L = 20, D = 256 random MPS, in FP64 and with BF16x3 contractions,
  against the FP64 oracle on the same input.  The results are compared in
  the canonical Schmidt gauge: per bond, the Schmidt values element by
  element (relative to the bond's largest), and the state distance from
  overlaps.  The smallest relative gap at a cut, (s_D - s_{D+1}) / s_1, is
  reported: the kept subspace moves by ~(perturbation) / gap.
* A truncated H|psi> at L = 6, N = 12, D = 16 against the oracle's tree sum,
  element by element on the dense 4096-vector.
* The Hartree-Fock-started FP64 Lanczos at L = 12, N = 48, D = 128 against
  the oracle's run of the same algorithm (fixture written by
  tests/golden/make_lanczos_L12_N48_D128.py, which calls only oracle/).
"""
import json
import os

import numpy as np
import pytest

import synth
from oracle import hamiltonian as OH
from oracle import lanczos as OL
from oracle import mps as M
from oracle import thc as TH

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def thck():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2409_12708_amd as p
    return p


def _rel_distance(a, b):
    aa, bb, ab = M.overlap(a, a), M.overlap(b, b), M.overlap(a, b)
    return np.sqrt(max(aa + bb - 2.0 * ab, 0.0)) / np.sqrt(bb)


def _schmidt_diff(a, b):
    """max over bonds of max_i |s_a,i - s_b,i| / s_b,1 (the shorter spectrum
    padded with zeros)."""
    sa, sb = M.schmidt_values(a), M.schmidt_values(b)
    worst = 0.0
    for x, y in zip(sa, sb):
        n = max(len(x), len(y))
        x = np.pad(x, (0, n - len(x)))
        y = np.pad(y, (0, n - len(y)))
        worst = max(worst, float(np.max(np.abs(x - y)) / y[0]))
    return worst


def _min_gap(spectra, D):
    gaps = [(s[D - 1] - s[D]) / s[0] for s in spectra if len(s) > D and s[0] > 0]
    return min(gaps) if gaps else None


@pytest.fixture(scope="module")
def l20_case():
    t, chi, zeta, sites = synth.make_workload("L20_N80_D256")
    sites = M.scale(sites, 1.0 / M.norm(sites))
    D = 256
    y = TH.spin_site_coeffs(chi[:, 0], 0)
    rec_l, rec_a = [], []
    lay = M.compress(M.apply_layer(sites, y, False), D, record=rec_l)
    add = M.compress(M.direct_sum([(1.0, lay), (1.0, sites)]), D, record=rec_a)
    return dict(t=t, chi=chi, zeta=zeta, sites=sites, y=y, D=D, lay=lay, add=add,
                gap_l=_min_gap(rec_l, D), gap_a=_min_gap(rec_a, D))


# Bars at L = 20, D = 256 (truncated at 25 of 39 bonds).  FP64: Schmidt values
# are perturbation-stable (|ds| <= ||dY||), ~1e-13 of s_1 per SVD, grown
# over the 39 sweep steps; the kept subspace moves by ~eps / gap, so the
# state distance is bounded through the smallest cut gap.  BF16x3: the
# absorb products carry ~2^-16 relative per product.
AT_SIZE = {"f64": (1e-10, 1e-6), "bf16x3": (1e-4, 1e-2)}


@pytest.mark.parametrize("prec", ["f64", "bf16x3"])
def test_layer_and_add_compress_at_L20_D256(thck, l20_case, prec):
    c = l20_case
    ctx = thck.Context(c["t"], c["chi"], c["zeta"])
    psi = thck.DeviceMPS.from_sites(c["sites"])
    st = thck.ThcStats()
    lay = ctx.apply_layer(psi, c["y"], False, c["D"], prec=prec, stats=st).to_sites()
    add = ctx.sum_compress([1.0, 1.0], [thck.DeviceMPS.from_sites(c["lay"]), psi], c["D"], prec=prec).to_sites()
    assert M.bonds(lay) == M.bonds(c["lay"])
    assert M.bonds(add) == M.bonds(c["add"])
    s_tol, d_tol = AT_SIZE[prec]
    for name, got, ref, gap in (("layer", lay, c["lay"], c["gap_l"]), ("add", add, c["add"], c["gap_a"])):
        ds = _schmidt_diff(got, ref)
        dist = _rel_distance(got, ref)
        print(f"L20 D256 {name}-compression prec={prec}: Schmidt values max diff {ds:.3e} (of s_1), "
              f"distance {dist:.3e}, smallest cut gap {gap:.3e}, SVD fallbacks {st.svd_fallbacks}")
        assert ds < s_tol
        assert dist < d_tol
    # the GPU output is right-canonical, as the library declares
    assert M.right_canonical_error(lay) < 1e-12


def test_apply_H_truncated_mid_size(thck):
    # L = 6 (12 sites), N = 12, D = 16 < the largest Schmidt rank 64: every
    # compression truncates; the oracle's tree sum in the same order
    L, N, D = 6, 12, 16
    rng = np.random.default_rng(70)
    t, chi, zeta = synth.thc_factors(rng, L, N)
    psi = synth.random_mps_tensors(rng, 2 * L, 64)
    psi = M.scale(psi, 1.0 / M.norm(psi))
    ctx = thck.Context(t, chi, zeta)
    st = thck.ThcStats()
    out = ctx.apply_H(thck.DeviceMPS.from_sites(psi), D=D, stats=st)
    ref_state = OH.apply_H(psi, t, chi, zeta, D=D, mode="tree")
    got, ref = M.to_dense(out.to_sites()), M.to_dense(ref_state)
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    print(f"truncated L6 N12 D16: rel err vs oracle tree {err:.3e}, discarded weight max "
          f"{st.discarded_weight_max:.3e}, SVD fallbacks {st.svd_fallbacks}")
    assert out.bond_list() == M.bonds(ref_state)
    assert err < 1e-8


def _lanczos_fixture():
    path = os.path.join(GOLDEN, "lanczos_L12_N48_D128.json")
    if not os.path.exists(path):
        return None
    return json.load(open(path))


# The Hartree-Fock-started run is spin-flip symmetric (spin-free H, closed
# shell), so at every bond between spatial orbitals the Schmidt values come
# in exactly degenerate pairs (pinned on the CPU in
# test_oracle_pins_lanczos.py).  While no bond reaches D the result is the
# unique untruncated one and the bar is 1e-8 relative on the lowest Ritz
# value.  Once bonds reach D a cut can fall inside a degenerate pair, where
# any vector of the pair is a correct truncation (reading A6): the oracle
# and the GPU may keep different ones, and their Krylov spaces drift apart
# from then on, by ~50x per truncated step (the Ritz values of steps 1, 2, 3
# agree to 3.9e-8, 2.4e-5, 1.1e-3).  The first two truncated steps are held
# to a sanity bound of 1e-3 on the Ritz value (the fixture holds more steps
# of the oracle's run, which the divergence makes incomparable), the
# degenerate pairs in the GPU's next Krylov vector are counted and reported,
# and what does not depend on the choice is checked exactly: the GPU's
# overlap matrix S equals the oracle's overlaps of the GPU's own Krylov
# vectors.
LANCZOS_EXACT, LANCZOS_TRUNCATED = 1e-8, 1e-3
LANCZOS_MAX_STEPS = 3


def test_lanczos_L12_N48_D128_from_hartree_fock(thck):
    fx = _lanczos_fixture()
    if fx is None or not fx["steps"]:
        pytest.skip("no oracle fixture")
    L, N, D, ne = fx["L"], fx["N"], fx["D"], fx["n_elec"]
    t, chi, zeta = synth.thc_factors(np.random.default_rng(fx["seed"]), L, N)
    hf = synth.occupation_mps_tensors(synth.hartree_fock_occupation(L, ne))
    steps = fx["steps"][:LANCZOS_MAX_STEPS]
    K = len(steps)
    ctx = thck.Context(t, chi, zeta)
    kr = thck.Krylov(ctx, thck.DeviceMPS.from_sites(hf), K, D=D)
    for s in steps:
        st = thck.ThcStats()
        g, tr, b = kr.step(st)
        rg = np.array(s["ritz_generalized"])
        e0 = abs(g[0] - rg[0]) / abs(rg[0])
        truncated = max(s["w_bonds"]) >= D or max(s["v_next_bonds"] or [1]) >= D
        print(f"L12 Lanczos step {s['i']}: lowest Ritz {g[0]:.12f} vs oracle {rg[0]:.12f} (rel {e0:.2e}), "
              f"beta {b:.6e} vs {s['beta']:.6e}, SVD second levels {st.svd_fallbacks}, max bond {st.max_bond}, "
              f"truncated {truncated}")
        if truncated:
            v = kr.vector(s["i"] + 1, D).to_sites()
            ties = sum(int(np.sum(np.abs(np.diff(x)) < 1e-10 * x[0]))
                       for bond, x in enumerate(M.schmidt_values(v), start=1) if bond % 2 == 0)
            print(f"  GPU v_{s['i'] + 1}: {ties} degenerate Schmidt pairs at the bonds between spatial orbitals")
        assert e0 < (LANCZOS_TRUNCATED if truncated else LANCZOS_EXACT)
        assert abs(b - s["beta"]) < (LANCZOS_TRUNCATED if truncated else 1e-8) * abs(s["beta"])
    # S_ij = <v_i|v_j> of the GPU's own Krylov vectors, by the oracle
    _, S = kr.matrices()
    vs = [kr.vector(i, D).to_sites() for i in range(K)]
    ref = np.array([[M.overlap(a, b) for b in vs] for a in vs])
    print(f"L12 Lanczos: max |S_gpu - S(oracle overlaps of the GPU vectors)| {np.abs(S - ref).max():.2e}")
    assert np.allclose(S, ref, rtol=0, atol=1e-12)
    kr.close()
