"""H|psi> with the THC-MPO (Sec. 3.2, Algorithm 1; App. D; Sec. 4.5).

Terms, in the order they enter the sum (readings A8, A10, A11):
* V terms (nu, s', mu, s) with nu outer, then s', mu, s; each is
  1/2 zeta_{mu nu} a+(chi^mu)_s a(chi^mu)_s a+(chi^nu)_s' a(chi^nu)_s' |psi>,
  built from the reused prefix |psi_{nu s'}> (Sec. 3.2, G factorisation) and
  scaled by 1/2 zeta on the prefix copy, as Algorithm 1 initialises it;
* T terms (i, s), i in ascending eigenvalue order of t, s = up, down;
  each is lam_i a+(u_i)_s a(u_i)_s |psi> (App. D), the scale put on the
  input copy; lam_i == 0 exactly is skipped.
Every layer application is followed by a compression (Fig. 4 arrows).
"""
from __future__ import annotations

import numpy as np

from . import mps as M
from .thc import kinetic_split, spin_site_coeffs, v_terms


def layer_compress(psi, x, sigma, dag, D, eps=M.CUTOFF):
    y = spin_site_coeffs(x, sigma)
    return M.compress(M.apply_layer(psi, y, dag), D, eps)


def one_body_pair(psi, x, sigma, D, eps=M.CUTOFF):
    """a+(x)_s a(x)_s |psi> as two compressed layers (annihilate first)."""
    t = layer_compress(psi, x, sigma, False, D, eps)
    return layer_compress(t, x, sigma, True, D, eps)


def prefix_states(psi, chi, D, eps=M.CUTOFF):
    """|psi_{nu s'}> = G_{nu s'}|psi> for all (nu, s') (Sec. 3.2 reuse)."""
    N = chi.shape[1]
    return {(nu, sp_): one_body_pair(psi, chi[:, nu], sp_, D, eps)
            for nu in range(N) for sp_ in (0, 1)}


def leaf_terms(psi, t, chi, zeta, D, eps=M.CUTOFF, include_T=True, include_V=True):
    """Generator of the compressed term states in summation order."""
    if include_V:
        N = chi.shape[1]
        pre = prefix_states(psi, chi, D, eps)
        for nu, sp_, mu, s in v_terms(N):
            c = 0.5 * zeta[mu, nu]
            if c == 0.0:
                continue
            start = M.scale(pre[nu, sp_], c)
            yield one_body_pair(start, chi[:, mu], s, D, eps)
    if include_T:
        lam, u = kinetic_split(t)
        for i in range(lam.shape[0]):
            if lam[i] == 0.0:
                continue
            for s in (0, 1):
                start = M.scale(psi, lam[i])
                yield one_body_pair(start, u[:, i], s, D, eps)


def add_compress(a, b, D, eps=M.CUTOFF):
    """compress(a (+) b), the MPS addition step of Algorithm 1."""
    return M.compress(M.direct_sum([(1.0, a), (1.0, b)]), D, eps)


def sum_sequential(leaves, D, eps=M.CUTOFF):
    """Algorithm 1: phi <- compress(phi + term) after every term."""
    phi = None
    for term in leaves:
        phi = term if phi is None else add_compress(phi, term, D, eps)
    return phi


def sum_tree(leaves, D, eps=M.CUTOFF, D_sum=None, D_final=None):
    """Pairwise reduction tree (Sec. 4.5, Fig. 11): pair (2k, 2k+1) at every
    level, an odd last element carries up unchanged (reading A8)."""
    Ds = D if D_sum is None else D_sum
    level = list(leaves)
    if not level:
        raise ValueError("empty sum")
    while len(level) > 1:
        nxt = [add_compress(level[2 * k], level[2 * k + 1], Ds, eps)
               for k in range(len(level) // 2)]
        if len(level) % 2:
            nxt.append(level[-1])
        level = nxt
    out = level[0]
    if D_final is not None and D_final != Ds:
        out = M.compress(out, D_final, eps)
    return out


def apply_H(psi, t, chi, zeta, D, mode="tree", eps=M.CUTOFF, include_T=True, include_V=True):
    """Compressed H|psi> with H = T + V (eq. 1, THC form eq. sum_of_H)."""
    leaves = leaf_terms(psi, t, chi, zeta, D, eps, include_T, include_V)
    if mode == "sequential":
        return sum_sequential(leaves, D, eps)
    if mode == "tree":
        return sum_tree(list(leaves), D, eps)
    raise ValueError(mode)


def sum_compress(coeffs, terms, D, eps=M.CUTOFF):
    """sum_i c_i |t_i>: each term scaled, then summed by the pairwise tree.

    With k = 1 this is compress(c_0 |t_0>)."""
    scaled = [M.scale(m, c) for c, m in zip(coeffs, terms)]
    if len(scaled) == 1:
        return M.compress(scaled[0], D, eps)
    return sum_tree(scaled, D, eps)
