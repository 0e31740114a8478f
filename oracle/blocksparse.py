"""Block-sparse MPS with abelian quantum numbers (N, 2 S_z): layers,
compression, direct sum and the compressed H|psi>.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's runs conserve the electron number and S_z, and Sec. 4.1 notes
that its MPS library stores site tensors block-sparse in these quantum
numbers to cut the cost.  This module is the oracle for that form: the same
compression as ``mps.compress`` (Fig. 3: right-canonical QR sweep, then SVDs
from left to right with the truncation rule of ``mps.truncation_rank``),
done block by block.  It must give the state the dense path gives.

Labels.  Sites are spin-orbitals j = 2p + s (s = 0 up, 1 down), as in
``fermion``.  Occupying site j adds (1, +1) for s = 0 and (1, -1) for s = 1 to
q = (N, 2 S_z).  Bond j sits left of site j (bond 0 and bond n are the
boundaries); its index space is a direct sum of sectors, one per label q,
listed as an ordered dict {q: dim}.  A site tensor is a dict
{(q_left, n): block} with block shape (dim of q_left, dim of q_right) and
q_right = q_left + delta(j, n): the tensor is zero outside these blocks.

Bond matrices are block-diagonal in these labels, so a factorisation of a
site matrix is a factorisation of each block: the LQ of the right sweep is
one LQ per left label, the SVD of the left sweep one SVD per right label,
and the truncation keeps the D largest singular values over all blocks of a
bond (the union of the blocks' spectra is the bond's spectrum).
"""
from __future__ import annotations

import numpy as np

from . import mps as M
from .fermion import C as C_, Z as Z_  # a = |0><1| on one site, and the Jordan-Wigner sign

CUTOFF = M.CUTOFF


def delta(j: int, n: int):
    """Quantum-number change of occupying (n = 1) site j."""
    if n == 0:
        return (0, 0)
    return (1, 1) if j % 2 == 0 else (1, -1)


def add(q, d):
    return (q[0] + d[0], q[1] + d[1])


# ---------------------------------------------------------------------------
# Construction and conversion
# ---------------------------------------------------------------------------

class BSMPS:
    """sites[j]: {(q_left, n): block}; bonds[j]: {q: dim} for j = 0..n."""

    def __init__(self, sites, bonds):
        self.sites = sites
        self.bonds = bonds

    @property
    def n(self):
        return len(self.sites)

    def copy(self):
        return BSMPS([{k: v.copy() for k, v in s.items()} for s in self.sites], [dict(b) for b in self.bonds])


def _reachable(n_sites, target):
    """Labels of bond j reachable from (0, 0) on the left that can still
    reach the target label on the right."""
    left = [{(0, 0)}]
    for j in range(n_sites):
        left.append({add(q, delta(j, x)) for q in left[-1] for x in (0, 1)})
    right = [None] * (n_sites + 1)
    right[n_sites] = {target}
    for j in range(n_sites - 1, -1, -1):
        right[j] = {q for q in left[j] for x in (0, 1) if add(q, delta(j, x)) in right[j + 1]}
    return [sorted(left[j] & right[j]) for j in range(n_sites + 1)]


def random_mps(rng, n_sites: int, n_elec: int, two_sz: int, D: int, dims=None) -> BSMPS:
    """A random state of fixed (N, 2 S_z), each sector of a bond of dimension
    min(D, dims(j, q)) (default: min(D, 3)), Gaussian blocks."""
    labels = _reachable(n_sites, (n_elec, two_sz))
    if not labels[n_sites]:
        raise ValueError("no state with these quantum numbers")
    bonds = []
    for j, qs in enumerate(labels):
        if j == 0 or j == n_sites:
            bonds.append({q: 1 for q in qs})
        else:
            bonds.append({q: min(D, dims(j, q) if dims else 3) for q in qs})
    sites = []
    for j in range(n_sites):
        s = {}
        for ql, dl in bonds[j].items():
            for x in (0, 1):
                qr = add(ql, delta(j, x))
                if qr in bonds[j + 1]:
                    s[(ql, x)] = rng.standard_normal((dl, bonds[j + 1][qr]))
        sites.append(s)
    return BSMPS(sites, bonds)


def from_occupation(occ) -> BSMPS:
    """The product state |occ> (one label, dimension 1, per bond)."""
    q = (0, 0)
    bonds = [{q: 1}]
    sites = []
    for j, x in enumerate(occ):
        qn = add(q, delta(j, int(x)))
        sites.append({(q, int(x)): np.ones((1, 1))})
        bonds.append({qn: 1})
        q = qn
    return BSMPS(sites, bonds)


def _offsets(bond):
    off, o = {}, 0
    for q, d in bond.items():
        off[q] = o
        o += d
    return off, o


def to_mps(bs: BSMPS):
    """Dense site tensors (left, 2, right), each bond's sectors in label order."""
    out = []
    for j, s in enumerate(bs.sites):
        lo, L = _offsets(bs.bonds[j])
        ro, R = _offsets(bs.bonds[j + 1])
        t = np.zeros((L, 2, R))
        for (ql, x), b in s.items():
            qr = add(ql, delta(j, x))
            t[lo[ql]:lo[ql] + b.shape[0], x, ro[qr]:ro[qr] + b.shape[1]] = b
        out.append(t)
    return out


def to_dense(bs: BSMPS) -> np.ndarray:
    return M.to_dense(to_mps(bs))


# ---------------------------------------------------------------------------
# Direct sum (Alg. 1's addition, block by block)
# ---------------------------------------------------------------------------

def direct_sum(terms) -> BSMPS:
    """sum_i c_i |psi_i> for states of one total label: each interior bond's
    sector q is the direct sum of the terms' sectors q; the coefficient goes
    on the first site, whose right bond is concatenated, and the last site's
    left bond is concatenated (the boundary bonds keep dimension 1)."""
    n = terms[0][1].n
    bonds = []
    for j in range(n + 1):
        if j == 0 or j == n:
            bonds.append(dict(terms[0][1].bonds[j]))
            continue
        b = {}
        for _, m in terms:
            for q, d in m.bonds[j].items():
                b[q] = b.get(q, 0) + d
        bonds.append(dict(sorted(b.items())))
    sites = []
    for j in range(n):
        s = {}
        # running offsets of each term inside every sector of bonds j and j + 1
        lo = {q: 0 for q in bonds[j]}
        ro = {q: 0 for q in bonds[j + 1]}
        for c, m in terms:
            for (ql, x), blk in m.sites[j].items():
                qr = add(ql, delta(j, x))
                key = (ql, x)
                if key not in s:
                    s[key] = np.zeros((bonds[j][ql], bonds[j + 1][qr]))
                r0 = 0 if j == 0 else lo[ql]
                c0 = 0 if j == n - 1 else ro[qr]
                v = c * blk if j == 0 else blk
                if j == 0 or j == n - 1:
                    # boundary sites: the dimension-1 side is shared, the
                    # other side is concatenated
                    if j == 0 and j == n - 1:
                        s[key] += v
                    elif j == 0:
                        s[key][:, c0:c0 + blk.shape[1]] = v
                    else:
                        s[key][r0:r0 + blk.shape[0], :] = v
                else:
                    s[key][r0:r0 + blk.shape[0], c0:c0 + blk.shape[1]] = v
            for q, d in m.bonds[j].items():
                if j > 0:
                    lo[q] += d
            for q, d in m.bonds[j + 1].items():
                if j + 1 < n:
                    ro[q] += d
        sites.append(s)
    return BSMPS(sites, bonds)


# ---------------------------------------------------------------------------
# Elementary layer (eq. elementary_MPO, App. C), block by block
# ---------------------------------------------------------------------------

def apply_layer(bs: BSMPS, y: np.ndarray, dag: bool) -> BSMPS:
    """sum_j y_j a_j (or a+_j) applied to the state, as ``mps.apply_layer``
    does with W_j = [[Z, y_j o], [0, I]], for y supported on sites of one
    spin (the THC layers act on one spin at a time), so that the operator
    changes the labels by one fixed d_op.

    MPO bond 0 (operator not yet applied, left of the site it acts on) keeps
    the ket's label q; MPO bond 1 (applied) shifts it to q + d_op.  Output
    sector r of an interior bond is the direct sum of the ket's sector r
    (MPO bond 0, first) and its sector r - d_op (MPO bond 1, second); the
    first bond keeps only MPO bond 0, the last only MPO bond 1."""
    n = bs.n
    supp = [j for j in range(n) if y[j] != 0.0]
    if not supp:
        raise ValueError("a layer with no coefficient")
    spins = {j % 2 for j in supp}
    if len(spins) != 1:
        raise ValueError("the layer must act on sites of one spin")
    dj = delta(supp[0], 1)
    dop = dj if dag else (-dj[0], -dj[1])
    # output bonds: (label) -> (dim, offset of the MPO-0 part, offset of the MPO-1 part)
    obonds, parts = [], []
    for j in range(n + 1):
        p0 = {q: d for q, d in bs.bonds[j].items()} if j < n else {}
        p1 = {add(q, dop): d for q, d in bs.bonds[j].items()} if j > 0 else {}
        labels = sorted(set(p0) | set(p1))
        dims, off = {}, {}
        for r in labels:
            d0, d1 = p0.get(r, 0), p1.get(r, 0)
            dims[r] = d0 + d1
            off[r] = (0, d0)
        obonds.append(dims)
        parts.append((p0, p1, off))
    o = C_T if dag else C_
    sites = []
    for j in range(n):
        s = {}
        _, _, offl = parts[j]
        _, _, offr = parts[j + 1]

        def put(lo_lab, m, lo_part, ro_lab, ro_part, blk):
            key = (lo_lab, m)
            if key not in s:
                s[key] = np.zeros((obonds[j][lo_lab], obonds[j + 1][ro_lab]))
            r0 = offl[lo_lab][lo_part]
            c0 = offr[ro_lab][ro_part]
            s[key][r0:r0 + blk.shape[0], c0:c0 + blk.shape[1]] += blk

        for (ql, x), blk in bs.sites[j].items():
            qr = add(ql, delta(j, x))
            if j < n - 1:  # MPO 0 -> 0: Z on the site (not on the last site)
                put(ql, x, 0, qr, 0, Z_[x, x] * blk)
            if j > 0:      # MPO 1 -> 1: identity (not on the first site)
                put(add(ql, dop), x, 1, add(qr, dop), 1, blk)
            for m in (0, 1):  # MPO 0 -> 1: y_j o on the site
                if y[j] != 0.0 and o[m, x] != 0.0:
                    put(ql, m, 0, add(qr, dop), 1, (y[j] * o[m, x]) * blk)
        sites.append(s)
    return BSMPS(sites, obonds)


C_T = C_.T


def layer_compress(bs: BSMPS, y: np.ndarray, dag: bool, D: int, eps: float = CUTOFF) -> BSMPS:
    """One leaf layer of the THC tree: apply, then compress (Fig. 3)."""
    return compress(apply_layer(bs, y, dag), D, eps)


# ---------------------------------------------------------------------------
# Compression (Fig. 3), block by block
# ---------------------------------------------------------------------------

def right_canonicalize(bs: BSMPS) -> BSMPS:
    """LQ sweep right -> left.  For site j and left label q, the rows of the
    site matrix X_q (left index) run over the sector q, its columns over
    (n, right index) for both occupations; X_q = L_q Q_q, Q_q replaces the
    blocks and L_q is absorbed into the blocks of site j - 1 that end in q."""
    out = bs.copy()
    for j in range(out.n - 1, 0, -1):
        s = out.sites[j]
        new_site, new_dims, Ls = {}, {}, {}
        for q, dl in out.bonds[j].items():
            parts = [(x, s[(q, x)]) for x in (0, 1) if (q, x) in s]
            if not parts:
                continue
            X = np.concatenate([b for _, b in parts], axis=1)  # (dl, sum of right dims)
            qq, rr = np.linalg.qr(X.T)  # X^T = Q R  <=>  X = R^T Q^T
            k = qq.shape[1]
            Qt = qq.T
            c = 0
            for x, b in parts:
                new_site[(q, x)] = Qt[:, c:c + b.shape[1]].copy()
                c += b.shape[1]
            new_dims[q] = k
            Ls[q] = rr.T  # (dl, k)
        out.sites[j] = new_site
        out.bonds[j] = new_dims
        prev = {}
        for (ql, x), b in out.sites[j - 1].items():
            qr = add(ql, delta(j - 1, x))
            if qr in Ls:
                prev[(ql, x)] = b @ Ls[qr]
        out.sites[j - 1] = prev
    return out


def svd_sweep(bs: BSMPS, D: int, eps: float = CUTOFF, record=None) -> BSMPS:
    """SVD truncation left -> right on a right-canonical block-sparse MPS.

    At bond j + 1 the site matrix Y_q for right label q stacks the blocks
    (q_left, n) with q_left + delta(j, n) = q (rows) over the sector q
    (columns).  Every Y_q is factorised; the bond keeps the k largest
    singular values of all blocks together, k = max(1, min(D, #{s > eps
    s_max})) as in the dense rule; U_q's kept columns replace the blocks,
    S V^T of the kept rows goes into site j + 1.  record, if given, receives
    each bond's full spectrum (all blocks, descending)."""
    out = bs.copy()
    for j in range(out.n - 1):
        s = out.sites[j]
        fac = {}
        for q in out.bonds[j + 1]:
            rows = [(key, b) for key, b in sorted(s.items()) if add(key[0], delta(j, key[1])) == q]
            if not rows:
                continue
            Y = np.concatenate([b for _, b in rows], axis=0)
            u, sv, vt = M.thin_svd(Y)
            fac[q] = (rows, u, sv, vt)
        allsv = np.sort(np.concatenate([f[2] for f in fac.values()]))[::-1] if fac else np.zeros(0)
        if record is not None:
            record.append(allsv.copy())
        k = M.truncation_rank(allsv, D, eps)
        # the k largest over all blocks (ties at the cut are the caller's to avoid)
        tagged = sorted(((v, q, i) for q, f in fac.items() for i, v in enumerate(f[2])), key=lambda t: -t[0])[:k]
        keep = {}
        for _, q, i in tagged:
            keep.setdefault(q, []).append(i)
        new_site, new_dims, carry = {}, {}, {}
        for q in out.bonds[j + 1]:
            if q not in keep:
                continue
            rows, u, sv, vt = fac[q]
            idx = sorted(keep[q])
            r0 = 0
            for key, b in rows:
                new_site[key] = u[r0:r0 + b.shape[0], idx].copy()
                r0 += b.shape[0]
            new_dims[q] = len(idx)
            carry[q] = sv[idx, None] * vt[idx]
        out.sites[j] = new_site
        out.bonds[j + 1] = new_dims
        nxt = {}
        for (ql, x), b in out.sites[j + 1].items():
            if ql in carry:
                nxt[(ql, x)] = carry[ql] @ b
        out.sites[j + 1] = nxt
    return out


def compress(bs: BSMPS, D: int, eps: float = CUTOFF, record=None) -> BSMPS:
    """Right-canonical sweep, then the truncating SVD sweep (as ``mps.compress``)."""
    return svd_sweep(right_canonicalize(bs), D, eps, record)


def svd_flops(bs: BSMPS):
    """(block, dense) flop counts of the SVD sweep's factorisations on this
    MPS's shapes, by the Golub-Reinsch model 4 m n^2 + 8 n^3 (m >= n) per
    factorised matrix: the cost the block form saves."""
    def gr(m, n):
        m, n = max(m, n), min(m, n)
        return 4.0 * m * n * n + 8.0 * n ** 3
    blk = dense = 0.0
    for j in range(bs.n - 1):
        rows_total = sum(bs.bonds[j].values()) * 2
        cols_total = sum(bs.bonds[j + 1].values())
        dense += gr(rows_total, cols_total)
        for q, dr in bs.bonds[j + 1].items():
            rows = sum(b.shape[0] for (ql, x), b in bs.sites[j].items() if add(ql, delta(j, x)) == q)
            if rows:
                blk += gr(rows, dr)
    return blk, dense


# ---------------------------------------------------------------------------
# H|psi> (eq. 1 in the THC form), block by block
# ---------------------------------------------------------------------------

def scale(bs: BSMPS, c: float) -> BSMPS:
    """c |psi>, carried by the last site (as ``mps.scale``)."""
    out = bs.copy()
    out.sites[-1] = {k: c * b for k, b in out.sites[-1].items()}
    return out


def one_body_pair(bs: BSMPS, x: np.ndarray, sigma: int, D: int, eps: float = CUTOFF) -> BSMPS:
    """a+(x)_sigma a(x)_sigma |psi> as two compressed layers (annihilate
    first), as ``hamiltonian.one_body_pair``; the label is unchanged."""
    from .thc import spin_site_coeffs
    y = spin_site_coeffs(x, sigma)
    return layer_compress(layer_compress(bs, y, False, D, eps), y, True, D, eps)


def apply_H(bs: BSMPS, t, chi, zeta, D: int, eps: float = CUTOFF) -> BSMPS:
    """Compressed H|psi> with the leaves of ``hamiltonian.leaf_terms`` (the
    prefix states G_{nu s'}|psi> of Sec. 3.2, then the second pair of each V
    term, then the kinetic pairs of App. D) summed by the pairwise tree of
    Sec. 4.5 (Fig. 11), every step block by block."""
    from .thc import kinetic_split, v_terms
    N = chi.shape[1]
    leaves = []
    pre = {(nu, sp_): one_body_pair(bs, chi[:, nu], sp_, D, eps) for nu in range(N) for sp_ in (0, 1)}
    for nu, sp_, mu, s in v_terms(N):
        c = 0.5 * zeta[mu, nu]
        if c == 0.0:
            continue
        leaves.append(one_body_pair(scale(pre[nu, sp_], c), chi[:, mu], s, D, eps))
    lam, u = kinetic_split(t)
    for i in range(lam.shape[0]):
        if lam[i] == 0.0:
            continue
        for s in (0, 1):
            leaves.append(one_body_pair(scale(bs, lam[i]), u[:, i], s, D, eps))
    level = leaves
    while len(level) > 1:
        nxt = [compress(direct_sum([(1.0, level[2 * k]), (1.0, level[2 * k + 1])]), D, eps)
               for k in range(len(level) // 2)]
        if len(level) % 2:
            nxt.append(level[-1])
        level = nxt
    return level[0]
