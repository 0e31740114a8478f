"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only draws random numbers and lays them out.  It holds none of
the method's arithmetic (no operator construction, no contraction, no
factorisation), so both the CPU oracle and the HIP path can consume exactly
the same inputs without sharing any code that computes a result.

Workload recipe (real arithmetic, numpy ``default_rng(seed)``, PCG64):

* draw order: ``t`` (L x L), ``chi`` (L x N), ``zeta`` (N x N), then the MPS
  site tensors for sites ``j = 0 .. n-1``;
* ``t`` and ``zeta``: a matrix A of iid N(0, 1) draws is symmetrised as
  ``triu(A) + triu(A, 1).T`` so that every entry is N(0, 1);
* ``chi``: iid N(0, 1/sqrt(L)) with 1/sqrt(L) read as the standard deviation,
  so that E ||chi^mu||^2 = 1;
* random MPS: ``n = 2L`` spin-orbital sites with local dimension 2 and bond
  profile ``min(2^j, 2^(n-j), D)``; entries iid N(0, 1), each site scaled by
  the constant 1/sqrt(2 * right_bond) so the state norm stays O(1).  The
  consumer normalises the state with its own norm routine;
* Hartree-Fock product state: bond dimension 1, the lowest ``n_elec/2``
  spatial orbitals doubly occupied (local basis index 0 = empty, 1 = occupied).

Site ``j = 2p + s`` holds spatial orbital ``p`` with spin ``s`` (0 = up,
1 = down).  Site tensors are float64 arrays laid out (left, phys, right),
row-major.
"""
from __future__ import annotations

import numpy as np

D_PHYS = 2


def sym_normal(rng: np.random.Generator, n: int) -> np.ndarray:
    """Symmetric n x n matrix whose entries are all N(0, 1)."""
    a = rng.standard_normal((n, n))
    return np.triu(a) + np.triu(a, 1).T


def thc_factors(rng: np.random.Generator, L: int, N: int):
    """Return (t, chi, zeta) drawn in that order."""
    t = sym_normal(rng, L)
    chi = rng.normal(0.0, 1.0 / np.sqrt(L), size=(L, N))
    zeta = sym_normal(rng, N)
    return t, chi, zeta


def bond_profile(n_sites: int, D: int) -> list[int]:
    """Bond dimensions b_0..b_n with b_j = min(2^j, 2^(n-j), D)."""
    out = []
    for j in range(n_sites + 1):
        out.append(int(min(2 ** min(j, 62), 2 ** min(n_sites - j, 62), D)))
    return out


def random_mps_tensors(rng: np.random.Generator, n_sites: int, D: int) -> list[np.ndarray]:
    """Un-normalised random real MPS site tensors (left, 2, right)."""
    b = bond_profile(n_sites, D)
    sites = []
    for j in range(n_sites):
        a = rng.standard_normal((b[j], D_PHYS, b[j + 1]))
        a *= 1.0 / np.sqrt(D_PHYS * b[j + 1])
        sites.append(a)
    return sites


def occupation_mps_tensors(occ: list[int]) -> list[np.ndarray]:
    """Bond-1 product state with site j in local state occ[j] (0 or 1)."""
    sites = []
    for o in occ:
        a = np.zeros((1, D_PHYS, 1))
        a[0, int(o), 0] = 1.0
        sites.append(a)
    return sites


def hartree_fock_occupation(L: int, n_elec: int) -> list[int]:
    """Closed-shell occupation: spatial orbitals 0..n_elec/2-1 doubly occupied."""
    if n_elec % 2 or n_elec < 0 or n_elec > 2 * L:
        raise ValueError("closed-shell occupation needs an even n_elec <= 2L")
    occ = [0] * (2 * L)
    for p in range(n_elec // 2):
        occ[2 * p] = 1
        occ[2 * p + 1] = 1
    return occ


def single_excitation_occupation(L: int, n_elec: int, spin: int = 0) -> list[int]:
    """The closed-shell occupation with one electron of the given spin moved
    from the highest occupied spatial orbital to the lowest empty one (an
    excited start vector orthogonal to the Hartree-Fock determinant)."""
    occ = hartree_fock_occupation(L, n_elec)
    homo, lumo = n_elec // 2 - 1, n_elec // 2
    if homo < 0 or lumo >= L:
        raise ValueError("no occupied or no empty orbital to excite")
    occ[2 * homo + spin] = 0
    occ[2 * lumo + spin] = 1
    return occ


def random_dense_vector(rng: np.random.Generator, n_sites: int) -> np.ndarray:
    """Random dense real vector of length 2^n_sites (un-normalised)."""
    return rng.standard_normal(2 ** n_sites)


# Workload table: the configurations the tests and the benchmark use.
WORKLOADS = {
    # dense 256x256 check, exact at D=16
    "L4_N8_D16": dict(L=4, N=8, D=16, seed=0),
    # untruncated at the full 512x1024 tile shapes (max Schmidt rank 2^8)
    "L8_N32_D256": dict(L=8, N=32, D=256, seed=0),
    # Lanczos ground state from Hartree-Fock, 12 electrons
    "L12_N48_D128": dict(L=12, N=48, D=128, seed=0, n_elec=12, krylov=20),
    # the throughput workload: 25,600 V terms + 40 T terms
    "L20_N80_D256": dict(L=20, N=80, D=256, seed=0),
}


def make_workload(name: str):
    """Return (t, chi, zeta, psi_sites) for a named random-MPS workload."""
    w = WORKLOADS[name]
    rng = np.random.default_rng(w["seed"])
    t, chi, zeta = thc_factors(rng, w["L"], w["N"])
    sites = random_mps_tensors(rng, 2 * w["L"], w["D"])
    return t, chi, zeta, sites
