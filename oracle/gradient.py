"""Gradient of E = <psi|H_THC|psi> with respect to the THC factors chi and
zeta (THC-factor fitting, Sec. 2.3; the G-term structure of Sec. 3.1).

With E_pq = sum_s a+_{ps} a_{qs} and the number-like operators
N_mu = sum_s a+(chi^mu)_s a(chi^mu)_s = sum_pq chi_p^mu chi_q^mu E_pq
(eq. G_mu_nu_def summed over the spins), V = 1/2 sum_{mu nu} zeta_{mu nu}
N_mu N_nu and, for a fixed real psi,

  dE/dzeta_{mu nu} = 1/2 <psi|N_mu N_nu|psi>            (all N^2 entries independent),
  dE/dchi_p^k      = 1/2 sum_nu (zeta_{k nu} + zeta_{nu k}) <psi|D_pk N_nu|psi>,
  D_pk = dN_k/dchi_p^k = sum_q chi_q^k (E_pq + E_qp).

T does not depend on chi or zeta.  Everything reduces to the transition
one-body matrices G^nu_pq = <psi|E_pq N_nu|psi>:
  <psi|N_mu N_nu|psi> = chi^mu^T G^nu chi^mu,
  <psi|D_pk N_nu|psi> = ((G^nu + G^nu^T) chi^k)_p.

Two implementations, pinned against each other and against finite
differences and a dense two-body density matrix in the tests:
* ``*_dense``: dense Fock-space vectors (n = 2L <= 16);
* ``*_mps``: the transition matrices from MPS contractions, with N_nu|psi>
  formed exactly by two layer applications per spin (no compression) and
  <psi|a+_i a_j|phi> read off by transfer-matrix chains with the
  Jordan-Wigner string of a+_i a_j.
"""
from __future__ import annotations

import numpy as np

from . import fermion as F
from . import mps as M
from .thc import spin_site_coeffs


# ---------------------------------------------------------------------------
# dense vectors
# ---------------------------------------------------------------------------

def number_like_dense(vec, chi, mu):
    """N_mu |vec> = sum_s a+(chi^mu)_s a(chi^mu)_s |vec> on a dense vector."""
    L = chi.shape[0]
    out = np.zeros_like(vec)
    for p in range(L):
        for q in range(L):
            c = chi[p, mu] * chi[q, mu]
            if c != 0.0:
                out += c * F.apply_E(vec, p, q, L)
    return out


def transition_1rdm_dense(bra, ket, L):
    """G_pq = <bra|E_pq|ket>."""
    return np.array([[bra @ F.apply_E(ket, p, q, L) for q in range(L)] for p in range(L)])


def energy_dense(vec, t, chi, zeta):
    """<vec|H|vec> with H of eq. (1) built from t and the THC factors."""
    L, N = chi.shape
    u = [number_like_dense(vec, chi, m) for m in range(N)]
    ev = 0.5 * sum(zeta[m, k] * (u[m] @ u[k]) for m in range(N) for k in range(N))
    et = sum(t[p, q] * (vec @ F.apply_E(vec, p, q, L)) for p in range(L) for q in range(L))
    return float(ev + et)


def transition_matrices_dense(vec, chi):
    """G^nu_pq = <vec|E_pq N_nu|vec> for every nu (N x L x L)."""
    L, N = chi.shape
    return np.stack([transition_1rdm_dense(vec, number_like_dense(vec, chi, nu), L) for nu in range(N)])


def gradient_from_transition(G, chi, zeta):
    """(dE/dchi (L x N), dE/dzeta (N x N)) from G^nu = <psi|E_pq N_nu|psi>."""
    L, N = chi.shape
    # <N_mu N_nu> = chi^mu^T G^nu chi^mu
    nn = np.array([[chi[:, m] @ G[nu] @ chi[:, m] for nu in range(N)] for m in range(N)])
    dzeta = 0.5 * nn
    zs = 0.5 * (zeta + zeta.T)
    dchi = np.zeros((L, N))
    for k in range(N):
        Mk = sum(zs[k, nu] * G[nu] for nu in range(N))
        dchi[:, k] = (Mk + Mk.T) @ chi[:, k]
    return dchi, dzeta


def gradient_dense(vec, chi, zeta):
    return gradient_from_transition(transition_matrices_dense(vec, chi), chi, zeta)


# ---------------------------------------------------------------------------
# MPS contractions
# ---------------------------------------------------------------------------

def number_like_spin_mps(psi, x, sigma):
    """a+(x)_s a(x)_s |psi> exactly: two layer applications, no compression
    (the bond grows by 4)."""
    y = spin_site_coeffs(x, sigma)
    return M.apply_layer(M.apply_layer(psi, y, False), y, True)


C_ANN = F.C            # c: |1> -> |0>
C_CRE = F.C.T          # c+: |0> -> |1>
ZDIAG = np.array([1.0, -1.0])


def _transfer(E, a, b, op=None):
    """sum_{s s'} op[s, s'] a[:, s, :]^T E b[:, s', :] (op = identity if None)."""
    if op is None:
        return np.einsum("ab,asc,bsd->cd", E, a, b)
    return np.einsum("ab,asc,st,btd->cd", E, a, op, b)


def transition_1rdm_mps(bra, ket):
    """g_ij = <bra|a+_i a_j|ket> for all spin-orbital sites i, j.

    a+_i a_j is c+_i Z_{i+1..j-1} c_j for i < j, c_j Z_{j+1..i-1} c+_i for
    i > j (no sign: the Jordan-Wigner strings to the left cancel) and c+c
    for i = j, so each entry is a transfer-matrix chain with one operator at
    each end and Z in between."""
    n = len(bra)
    Zop = np.diag(ZDIAG)
    left = [np.ones((1, 1))]
    for j in range(n):
        left.append(_transfer(left[-1], bra[j], ket[j]))
    right = [np.ones((1, 1))]
    for j in range(n - 1, -1, -1):
        right.append(np.einsum("asc,bsd,cd->ab", bra[j], ket[j], right[-1]))
    right = right[::-1]  # right[j] covers sites j..n-1; right[n] = [[1]]
    g = np.zeros((n, n))
    for i in range(n):
        g[i, i] = np.sum(_transfer(left[i], bra[i], ket[i], C_CRE @ C_ANN) * right[i + 1])
        for op_l, op_r, sign_pos in ((C_CRE, C_ANN, 0), (C_ANN, C_CRE, 1)):
            O = _transfer(left[i], bra[i], ket[i], op_l)
            for j in range(i + 1, n):
                val = np.sum(_transfer(O, bra[j], ket[j], op_r) * right[j + 1])
                if sign_pos == 0:
                    g[i, j] = val      # a+_i a_j, i < j
                else:
                    g[j, i] = val      # a+_j a_i, j > i
                O = _transfer(O, bra[j], ket[j], Zop)
    return g


def spin_summed(g, L):
    """G_pq = sum_s g_{2p+s, 2q+s}."""
    return g[0::2, 0::2] + g[1::2, 1::2]


def transition_matrices_mps(psi, chi):
    """G^nu_pq = <psi|E_pq N_nu|psi> from N_nu|psi> = sum_s' n_{nu s'}|psi>."""
    L, N = chi.shape
    out = np.zeros((N, L, L))
    for nu in range(N):
        for sp_ in (0, 1):
            phi = number_like_spin_mps(psi, chi[:, nu], sp_)
            out[nu] += spin_summed(transition_1rdm_mps(psi, phi), L)
    return out


def energy_mps(psi, t, chi, zeta):
    """<psi|H|psi> from the same transition matrices: 1/2 sum zeta <N_mu N_nu>
    + sum t_pq <E_pq>."""
    L, N = chi.shape
    G = transition_matrices_mps(psi, chi)
    nn = np.array([[chi[:, m] @ G[nu] @ chi[:, m] for nu in range(N)] for m in range(N)])
    g1 = spin_summed(transition_1rdm_mps(psi, psi), L)
    return float(0.5 * np.sum(zeta * nn) + np.sum(t * g1))


def gradient_mps(psi, chi, zeta):
    return gradient_from_transition(transition_matrices_mps(psi, chi), chi, zeta)
