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
    """Compressed H|psi> with H = T + V (eq. 1, THC form eq. sum_of_H).

    mode "sequential": Algorithm 1's running sum; "tree": the pairwise tree
    of Fig. 11 over all terms; "two_trees": the terms split by nu into the V
    terms with nu < N/2 and the rest (V terms with nu >= N/2, then T), each
    part summed by its own tree and the two sums added (reading R13, the
    order of the GPU's two-stream application)."""
    leaves = leaf_terms(psi, t, chi, zeta, D, eps, include_T, include_V)
    if mode == "sequential":
        return sum_sequential(leaves, D, eps)
    if mode == "tree":
        return sum_tree(list(leaves), D, eps)
    if mode == "two_trees":
        leaves = list(leaves)
        N = chi.shape[1]
        n_v = [0, 0]  # V terms with nu < N/2, with nu >= N/2
        if include_V:
            for nu, sp_, mu, s in v_terms(N):
                if zeta[mu, nu] != 0.0:
                    n_v[nu >= N // 2] += 1
        n_first = n_v[0]
        if n_v[0] == 0 or n_v[1] == 0:  # one part without V terms: the single tree
            return sum_tree(leaves, D, eps)
        return add_compress(sum_tree(leaves[:n_first], D, eps), sum_tree(leaves[n_first:], D, eps), D, eps)
    raise ValueError(mode)


def sum_compress(coeffs, terms, D, eps=M.CUTOFF):
    """sum_i c_i |t_i>: each term scaled, then summed by the pairwise tree.

    With k = 1 this is compress(c_0 |t_0>)."""
    scaled = [M.scale(m, c) for c, m in zip(coeffs, terms)]
    if len(scaled) == 1:
        return M.compress(scaled[0], D, eps)
    return sum_tree(scaled, D, eps)


# ---------------------------------------------------------------------------
# The same tree, fed one node at a time, and H|psi> with its independent
# compressions handed to a caller-supplied map (large cases only).
# ---------------------------------------------------------------------------

class StreamTree:
    """The pairwise tree of ``sum_tree`` built as the nodes arrive.

    Nodes reaching a level in order pair as (2k, 2k+1): the first two nodes
    waiting at a level are compressed together and the result moves up one
    level.  ``finish`` carries a lone node up, lowest level first, as the odd
    last element of a level carries up in ``sum_tree`` (Sec. 4.5, Fig. 11).
    The pairs and their operands are those of ``sum_tree``; only the time at
    which each pair is formed differs.  ``push(node, level)`` with level > 0
    enters the root of a complete subtree of 2**level consecutive leaves.
    """

    def __init__(self, D, eps=M.CUTOFF):
        self.D, self.eps = D, eps
        self.levels = []

    def push(self, node, level=0):
        while len(self.levels) <= level:
            self.levels.append([])
        self.levels[level].append(node)
        if len(self.levels[level]) == 2:
            a, b = self.levels[level]
            self.levels[level] = []
            self.push(add_compress(a, b, self.D, self.eps), level + 1)

    def finish(self):
        while True:
            filled = [l for l, q in enumerate(self.levels) if q]
            if not filled:
                raise ValueError("empty sum")
            if len(filled) == 1:
                return self.levels[filled[0]][0]
            low = filled[0]
            node = self.levels[low].pop()
            self.push(node, low + 1)


def _leaf_job(args):
    start, x, s, D, eps = args
    return one_body_pair(start, x, s, D, eps)


def _pair_job(args):
    a, b, D, eps = args
    return add_compress(a, b, D, eps)


def apply_H_mapped(psi, t, chi, zeta, D, eps=M.CUTOFF, mapper=map, window=256):
    """``apply_H(mode="tree")`` with the independent compressions handed to
    ``mapper`` (the builtin ``map``, or a process pool's ordered ``map``).

    The prefix states, the leaves and the pairs of the tree are the ones of
    ``apply_H``: leaves are produced in summation order in windows of
    ``window`` (a power of two) consecutive leaves; a full window starts at
    a multiple of ``window``, so its leaves form a complete subtree of the
    tree, reduced level by level (each level's pairs through ``mapper``) and
    entered at its level; the leaves of a last, partial window are entered
    one by one.  Only the schedule differs from ``apply_H``.
    """
    if window < 1 or window & (window - 1):
        raise ValueError("window must be a power of two")
    depth = window.bit_length() - 1
    N = chi.shape[1]
    pre_specs = [(psi, chi[:, nu], sp_, D, eps) for nu in range(N) for sp_ in (0, 1)]
    pre_states = list(mapper(_leaf_job, pre_specs))
    pre = {(nu, sp_): pre_states[2 * nu + sp_] for nu in range(N) for sp_ in (0, 1)}
    specs = []
    for nu, sp_, mu, s in v_terms(N):
        c = 0.5 * zeta[mu, nu]
        if c != 0.0:
            specs.append(((nu, sp_), c, chi[:, mu], s))
    lam, u = kinetic_split(t)
    for i in range(lam.shape[0]):
        if lam[i] != 0.0:
            for s in (0, 1):
                specs.append((None, lam[i], u[:, i], s))
    tree = StreamTree(D, eps)
    for w0 in range(0, len(specs), window):
        chunk = specs[w0:w0 + window]
        jobs = [(M.scale(psi if key is None else pre[key], c), x, s, D, eps) for key, c, x, s in chunk]
        level = list(mapper(_leaf_job, jobs))
        if len(chunk) == window:
            for _ in range(depth):
                level = list(mapper(_pair_job, [(level[2 * k], level[2 * k + 1], D, eps)
                                                for k in range(len(level) // 2)]))
            tree.push(level[0], depth)
        else:
            for node in level:
                tree.push(node, 0)
    return tree.finish()
