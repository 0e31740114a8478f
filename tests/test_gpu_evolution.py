"""GPU parity of the Krylov time evolution (Sec. 2.2: psi(t + delta) =
sum_i a_i v_i with a(delta) = exp(-i delta H~) a(0); App. A) against the
FP64 oracle's run of the same algorithm (``oracle.evolution``) and, where
the Krylov space is exhausted or one-dimensional, against the dense
exponential of eq. (1).  Complex states are (re, im) pairs of real MPS on
both sides; instances of different L, N and D run in one call.
"""
import numpy as np
import pytest
import scipy.linalg
import scipy.sparse.linalg

import synth
from oracle import evolution as EV
from oracle import fermion as F
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


def _dense(pair):
    re, im = pair
    return M.to_dense(re.to_sites()) + 1j * M.to_dense(im.to_sites())


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _random_start(rng, n, D):
    psi = synth.random_mps_tensors(rng, n, D)
    return M.scale(psi, 1.0 / M.norm(psi))


def test_exhausted_krylov_space_is_the_dense_exponential(thck):
    # L = 2 (16 states), K = 16: the step is exact, so it must equal
    # expm(-i delta H) psi of the dense H of eq. (1); two steps, so the
    # second starts from a complex state
    rng = np.random.default_rng(21)
    t, chi, zeta = synth.thc_factors(rng, 2, 3)
    psi = _random_start(rng, 4, 4)
    ctx = thck.Context(t, chi, zeta)
    (out,), dims = thck.evolve([(ctx, thck.DeviceMPS.from_sites(psi), None, 4)], K=16, delta=0.2, n_steps=2)
    H = F.hamiltonian_sparse(t, TH.thc_v(chi, zeta)).toarray()
    want = scipy.linalg.expm(-0.4j * H) @ M.to_dense(psi)
    print("krylov dims", dims.tolist(), "err", _rel(_dense(out), want))
    assert _rel(_dense(out), want) < 1e-11
    assert (dims <= 16).all()


def test_eigenstate_gains_a_phase(thck):
    # breakdown after one vector: psi(delta) = exp(-i E delta) psi
    rng = np.random.default_rng(22)
    t, chi, zeta = synth.thc_factors(rng, 2, 3)
    H = F.hamiltonian_sparse(t, TH.thc_v(chi, zeta)).toarray()
    w, U = np.linalg.eigh(H)
    psi = _dense_to_mps(U[:, 3], 4)
    ctx = thck.Context(t, chi, zeta)
    (out,), dims = thck.evolve([(ctx, thck.DeviceMPS.from_sites(psi), None, 4)], K=5, delta=0.9, n_steps=1)
    assert dims.tolist() == [[1]]
    assert _rel(_dense(out), np.exp(-0.9j * w[3]) * U[:, 3]) < 1e-12


@pytest.mark.parametrize("prec,tol", [("f64", 1e-12), ("f32", 1e-5), ("bf16x3", 1e-3)])
def test_untruncated_evolution_matches_oracle(thck, prec, tol):
    # L = 3 at D = 8 keeps every Schmidt value; K = 6, two steps of 0.1
    rng = np.random.default_rng(23)
    t, chi, zeta = synth.thc_factors(rng, 3, 4)
    psi = _random_start(rng, 6, 8)
    ctx = thck.Context(t, chi, zeta)
    (out,), dims = thck.evolve([(ctx, thck.DeviceMPS.from_sites(psi), None, 8, {"prec": prec})], K=6, delta=0.1,
                               n_steps=2)
    ref, rdims = EV.evolve((psi, None), t, chi, zeta, 8, 6, 0.1, 2)
    err = _rel(_dense(out), EV.to_dense_complex(ref))
    print(prec, "dims", dims.tolist(), rdims, "err vs oracle", err)
    assert dims[0].tolist() == rdims
    assert err < tol
    if prec != "f64":
        assert err > 1e-13  # the reduced-precision contractions really ran


def test_truncated_uneven_instances_match_oracle(thck):
    # three instances of uneven size in one call: L = 3, 4, 5 (N = 4, so the
    # oracle finishes in seconds) at D = 4, 8, 8, below each one's largest
    # Schmidt rank (8, 16, 32), so the middle bonds truncate; generic random
    # starts (no degenerate Schmidt values at the cuts), K = 4, two steps of
    # 0.05
    rng = np.random.default_rng(24)
    cases = []
    for L, D in ((3, 4), (4, 8), (5, 8)):
        t, chi, zeta = synth.thc_factors(rng, L, 4)
        cases.append((t, chi, zeta, _random_start(rng, 2 * L, D), D))
    ctxs = [thck.Context(t, chi, zeta) for t, chi, zeta, _, _ in cases]
    insts = [(c, thck.DeviceMPS.from_sites(p), None, D) for c, (_, _, _, p, D) in zip(ctxs, cases)]
    outs, dims = thck.evolve(insts, K=4, delta=0.05, n_steps=2)
    for q, ((t, chi, zeta, psi, D), out) in enumerate(zip(cases, outs)):
        ref, rdims = EV.evolve((psi, None), t, chi, zeta, D, 4, 0.05, 2)
        err = _rel(_dense(out), EV.to_dense_complex(ref))
        print("instance", q, "L", len(psi) // 2, "D", D, "dims", dims[q].tolist(), "err vs oracle", err)
        assert dims[q].tolist() == rdims
        assert err < 1e-9


def test_hartree_fock_single_excitation_start(thck):
    # the time-evolution configuration's start vector: one electron of spin
    # up moved from the highest occupied to the lowest empty orbital of the
    # closed-shell determinant (Sec. 4 starts its run from a_{3,up}|psi_0>);
    # L = 4 with 4 electrons, untruncated at D = 16, against the oracle and
    # the dense exponential within the Krylov error bound of App. A
    L = 4
    rng = np.random.default_rng(25)
    t, chi, zeta = synth.thc_factors(rng, L, 4)
    psi = synth.occupation_mps_tensors(synth.single_excitation_occupation(L, 4))
    ctx = thck.Context(t, chi, zeta)
    (out,), dims = thck.evolve([(ctx, thck.DeviceMPS.from_sites(psi), None, 16)], K=8, delta=0.05, n_steps=2)
    ref, rdims = EV.evolve((psi, None), t, chi, zeta, 16, 8, 0.05, 2)
    got = _dense(out)
    assert dims[0].tolist() == rdims
    assert _rel(got, EV.to_dense_complex(ref)) < 1e-12
    H = F.hamiltonian_sparse(t, TH.thc_v(chi, zeta))
    want = scipy.sparse.linalg.expm_multiply(-0.1j * H, M.to_dense(psi).astype(complex))
    assert _rel(got, want) < 1e-8
    assert abs(np.linalg.norm(got) - 1.0) < 1e-12


def test_evolve_rejects_bad_arguments(thck):
    rng = np.random.default_rng(26)
    t, chi, zeta = synth.thc_factors(rng, 2, 3)
    ctx = thck.Context(t, chi, zeta)
    psi = thck.DeviceMPS.from_sites(_random_start(rng, 4, 4))
    with pytest.raises(thck.ThcError) as e:
        thck.evolve([(ctx, psi, None, 4)], K=17, delta=0.1, n_steps=1)
    assert e.value.status == -1
    zero = thck.DeviceMPS.from_sites([np.zeros((1, 2, 1))] * 4)
    with pytest.raises(thck.ThcError) as e:
        thck.evolve([(ctx, zero, None, 4)], K=4, delta=0.1, n_steps=1)
    assert e.value.status == -1


def test_complex_start_and_degenerate_calls(thck):
    # a start with both parts given (a genuinely complex state), K = 1 (a
    # phase from <H>), and n_steps = 0 (the input comes back unchanged)
    rng = np.random.default_rng(27)
    t, chi, zeta = synth.thc_factors(rng, 3, 4)
    re = _random_start(rng, 6, 8)
    im = M.scale(_random_start(rng, 6, 8), 0.5)
    ctx = thck.Context(t, chi, zeta)
    dre, dim = thck.DeviceMPS.from_sites(re), thck.DeviceMPS.from_sites(im)
    for K, steps in ((3, 2), (1, 1)):
        (out,), dims = thck.evolve([(ctx, dre, dim, 8)], K=K, delta=0.07, n_steps=steps)
        ref, rdims = EV.evolve((re, im), t, chi, zeta, 8, K, 0.07, steps)
        err = _rel(_dense(out), EV.to_dense_complex(ref))
        print("K", K, "dims", dims.tolist(), rdims, "err vs oracle", err)
        assert dims[0].tolist() == rdims
        assert err < 1e-12
    (out,), dims = thck.evolve([(ctx, dre, dim, 8)], K=4, delta=0.07, n_steps=0)
    assert dims.shape == (1, 0)
    want = M.to_dense(re) + 1j * M.to_dense(im)
    assert _rel(_dense(out), want) < 1e-15


def test_complex_sum_compress_and_overlap_match_oracle(thck):
    # the complex combination and overlap entry points on (re, im) pairs with
    # absent parts, untruncated (D = 8 at L = 3) and truncated (D = 4)
    rng = np.random.default_rng(28)
    t, chi, zeta = synth.thc_factors(rng, 3, 4)
    ctx = thck.Context(t, chi, zeta)
    xs = [(_random_start(rng, 6, 8), _random_start(rng, 6, 8)), (_random_start(rng, 6, 8), None),
          (None, _random_start(rng, 6, 8))]
    coeffs = [0.3 - 0.7j, 1.1 + 0.2j, -0.4j]
    dev = [tuple(None if p is None else thck.DeviceMPS.from_sites(p) for p in x) for x in xs]
    for D, tol in ((8, 1e-12), (4, 1e-9)):
        got = ctx.sum_compress_complex(coeffs, dev, D)
        ref = EV.ccombine(coeffs, xs, D)
        err = _rel(_dense(got), EV.to_dense_complex(ref))
        print("D", D, "err vs oracle", err)
        assert err < tol
    for a, b in ((0, 2), (0, 1), (1, 2), (2, 0)):
        got = ctx.overlap_complex(dev[a], dev[b])
        want = EV.coverlap(xs[a], xs[b])
        assert abs(got - want) < 1e-13, (a, b, got, want)
    # a real combination of real states: the imaginary output is the zero MPS
    re, im = ctx.sum_compress_complex([2.0], [dev[1]], 8)
    assert im.bond_list() == [1] * 7 and not im.to_sites()[0].any()
    assert _rel(M.to_dense(re.to_sites()), 2.0 * M.to_dense(xs[1][0])) < 1e-12
