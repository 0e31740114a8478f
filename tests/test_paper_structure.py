"""The oracle against structural facts the paper states (tests/golden/paper_structure.txt).

CPU only.  The fixture holds the values as the paper gives them, each with its
section; these tests check the oracle's layer MPO, term table and reduction
tree against them.
"""
import math
import os

import numpy as np
import pytest

from oracle import hamiltonian as H
from oracle import mps as M
from oracle import thc as TH

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "paper_structure.txt")


def _facts():
    out = {}
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        key, val = line.split()
        out[key] = int(val)
    return out


FACTS = _facts()


@pytest.mark.parametrize("n", [2, 5, 9])
@pytest.mark.parametrize("dag", [False, True])
def test_layer_mpo_bond_dimension(n, dag):
    y = np.random.default_rng(n).standard_normal(n)
    ws = M.layer_mpo(y, dag)
    assert len(ws) == n
    D = FACTS["layer_bond_dimension"]
    # boundary sites keep one row / one column; every inner bond is D
    assert ws[0].shape[0] == 1 and ws[-1].shape[1] == 1
    for a, b in zip(ws[:-1], ws[1:]):
        assert a.shape[1] == b.shape[0] == D


def test_layer_application_doubles_the_bond():
    rng = np.random.default_rng(3)
    n, chi = 6, 4
    psi = [rng.standard_normal((1 if j == 0 else chi, 2, 1 if j == n - 1 else chi)) for j in range(n)]
    out = M.apply_layer(psi, rng.standard_normal(n), dag=False)
    g = FACTS["layer_bond_growth"]
    for j in range(1, n):
        assert out[j].shape[0] == g * psi[j].shape[0]
        assert out[j - 1].shape[2] == g * psi[j - 1].shape[2]


@pytest.mark.parametrize("N", [1, 3, 4, 7])
def test_coulomb_subterm_count(N):
    terms = list(TH.v_terms(N))
    assert len(terms) == FACTS["coulomb_subterms_per_rank_squared"] * N * N
    assert len(set(terms)) == len(terms)  # each (nu, s', mu, s) once


@pytest.mark.parametrize("N", [1, 2, 4, 8])
def test_reduction_tree_additions_and_levels(N, monkeypatch):
    # count the addition-compressions and the depth of the oracle's tree on
    # 4 N^2 leaves; a stand-in addition records the depth of each node
    k = FACTS["coulomb_subterms_per_rank_squared"] * N * N
    calls = []

    def fake_add(a, b, D, eps):
        calls.append((a, b))
        return max(a, b) + 1

    monkeypatch.setattr(H, "add_compress", fake_add)
    depth = H.sum_tree([0] * k, D=1)
    assert len(calls) == k + FACTS["additions_minus_subterms"]
    assert depth == FACTS["reduction_levels_per_log2_rank"] * int(math.log2(N)) + FACTS["reduction_levels_offset"]


@pytest.mark.parametrize("k", [3, 5, 6, 7, 33])
def test_reduction_tree_any_count(k, monkeypatch):
    # counts that are not powers of two: k - 1 additions and ceil(log2 k)
    # levels, the odd node carried up
    calls = []
    monkeypatch.setattr(H, "add_compress", lambda a, b, D, eps: calls.append(1) or max(a, b) + 1)
    assert H.sum_tree([0] * k, D=1) == math.ceil(math.log2(k))
    assert len(calls) == k - 1
