"""GPU parity of the two-stream H application (THC_FLAG_TWO_STREAMS): the V
terms split by nu into two halves, each summed by its own pairwise tree on
its own stream and host thread, the two sums added (reading R13; the
oracle's "two_trees" order).  Untruncated it is eq. (1) applied densely;
truncated it matches the oracle's two-tree sum; inside Lanczos and time
evolution the flag flows through the H applications.
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


@pytest.fixture(scope="module")
def thck():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2409_12708_amd as p
    return p


def _norm_mps(rng, n, D):
    psi = synth.random_mps_tensors(rng, n, D)
    return M.scale(psi, 1.0 / M.norm(psi))


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_two_streams_untruncated_is_dense_eq1(thck):
    rng = np.random.default_rng(40)
    t, chi, zeta, sites = synth.make_workload("L4_N8_D16")
    psi = M.scale(sites, 1.0 / M.norm(sites))
    ctx = thck.Context(t, chi, zeta)
    d = thck.DeviceMPS.from_sites(psi)
    st2, st1 = thck.ThcStats(), thck.ThcStats()
    out = ctx.apply_H(d, D=16, stats=st2, flags=thck.FLAG_TWO_STREAMS)
    one = ctx.apply_H(d, D=16, stats=st1)
    want = F.apply_H_dense(M.to_dense(psi), t, TH.thc_v(chi, zeta))
    got = M.to_dense(out.to_sites())
    print("two streams vs dense", _rel(got, want))
    assert _rel(got, want) < 1e-12
    assert _rel(got, M.to_dense(one.to_sites())) < 1e-12
    # the same terms: a tree over k leaves and two trees plus their sum both take k - 1 additions
    assert st2.n_compressions == st1.n_compressions


@pytest.mark.parametrize("L,N,D", [(4, 6, 8), (5, 7, 8)])
def test_two_streams_truncated_matches_oracle_two_trees(thck, L, N, D):
    # truncated (D below the largest Schmidt rank), odd and even N: the
    # mode-matched oracle order
    rng = np.random.default_rng(41 + N)
    t, chi, zeta = synth.thc_factors(rng, L, N)
    psi = _norm_mps(rng, 2 * L, 16)
    ctx = thck.Context(t, chi, zeta)
    out = ctx.apply_H(thck.DeviceMPS.from_sites(psi), D=D, flags=thck.FLAG_TWO_STREAMS)
    ref = M.to_dense(OH.apply_H(psi, t, chi, zeta, D=D, mode="two_trees"))
    err = _rel(M.to_dense(out.to_sites()), ref)
    print(f"truncated L{L} N{N} D{D}: rel err vs oracle two trees {err:.3e}")
    assert err < 1e-8


def test_two_streams_lanczos_untruncated(thck):
    # three untruncated Lanczos steps with and without the flag give the same
    # Ritz values (and the oracle's)
    L, N, K = 3, 4, 3
    t, chi, zeta = synth.thc_factors(np.random.default_rng(16), L, N)
    psi = _norm_mps(np.random.default_rng(43), 2 * L, 8)
    ctx = thck.Context(t, chi, zeta)
    runs = []
    for flags in (0, thck.FLAG_TWO_STREAMS):
        kr = thck.Krylov(ctx, thck.DeviceMPS.from_sites(psi), K, D=8, flags=flags)
        runs.append([kr.step()[0] for _ in range(K)])
        kr.close()
    st = OL.KrylovState(psi, K)
    ref = [OL.krylov_step(st, t, chi, zeta, 8)[0] for _ in range(K)]
    for a, b, r in zip(*runs, ref):
        assert np.allclose(a, b, rtol=1e-12, atol=1e-12)
        assert np.allclose(b, r, rtol=1e-10, atol=1e-10)


def test_two_streams_in_time_evolution(thck):
    # the flag reaches the H applications of krylov_evolve (untruncated: the
    # same state as without it)
    rng = np.random.default_rng(44)
    t, chi, zeta = synth.thc_factors(rng, 3, 4)
    psi = _norm_mps(rng, 6, 8)
    ctx = thck.Context(t, chi, zeta)
    res = []
    for flags in (0, thck.FLAG_TWO_STREAMS):
        (out,), _ = thck.evolve([(ctx, thck.DeviceMPS.from_sites(psi), None, 8, {"flags": flags})], K=4,
                                delta=0.1, n_steps=1)
        res.append(M.to_dense(out[0].to_sites()) + 1j * M.to_dense(out[1].to_sites()))
    assert _rel(res[1], res[0]) < 1e-12
