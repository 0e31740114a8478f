"""GPU tests of the captured launch sequences (THC_FLAG_GRAPHS) and of the
GEMM tile autotuner: replays of captured compression batches give the
eager results bit for bit, with eager work and synchronisations between the
replays, and every replay is checked."""
import numpy as np
import pytest

import synth
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


@pytest.mark.parametrize("L,N,D,Dpsi", [(4, 8, 16, 16), (6, 6, 8, 32)])
def test_graph_replays_match_eager(thck, L, N, D, Dpsi):
    import torch
    rng = np.random.default_rng(80 + L)
    t, chi, zeta = synth.thc_factors(rng, L, N)
    psi = synth.random_mps_tensors(rng, 2 * L, Dpsi)
    psi = M.scale(psi, 1.0 / M.norm(psi))
    ctx = thck.Context(t, chi, zeta)
    d = thck.DeviceMPS.from_sites(psi)
    eager = ctx.apply_H(d, D=D).to_sites()
    replays = 0
    for rep in range(4):
        st = thck.ThcStats()
        out = ctx.apply_H(d, D=D, stats=st, flags=thck.FLAG_GRAPHS).to_sites()
        replays += st.graph_replays
        print(f"L={L} D={D} graph call {rep}: captures {st.graph_captures}, replays {st.graph_replays}")
        assert M.bonds(out) == M.bonds(eager)
        for a, b in zip(out, eager):
            assert np.array_equal(a, b), rep
        # eager work and a synchronisation between the replays
        ctx.overlap(d, d)
        ctx.compress(d, D=D)
        torch.cuda.synchronize()
    assert replays > 0
    if L == 4:
        ref = F.apply_H_dense(M.to_dense(psi), t, TH.thc_v(chi, zeta))
        got = M.to_dense(eager)
        assert np.linalg.norm(got - ref) < 1e-12 * np.linalg.norm(ref)


def test_graph_replays_in_lanczos(thck):
    # a Krylov run with graphs equals the run without, step by step
    L, N = 3, 4
    t, chi, zeta = synth.thc_factors(np.random.default_rng(16), L, N)
    hf = synth.occupation_mps_tensors(synth.hartree_fock_occupation(L, 2))
    ctx = thck.Context(t, chi, zeta)
    a = thck.Krylov(ctx, thck.DeviceMPS.from_sites(hf), 4, D=8)
    b = thck.Krylov(ctx, thck.DeviceMPS.from_sites(hf), 4, D=8, flags=thck.FLAG_GRAPHS)
    for i in range(4):
        ga, _, ba = a.step()
        gb, _, bb = b.step()
        assert np.array_equal(ga, gb) and ba == bb, i
