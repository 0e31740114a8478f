"""MPS primitives of the oracle (Sec. 2.1, Fig. 3; Sec. 3.1; App. C).

An MPS is a Python list of float64 site tensors shaped (left, 2, right),
bond 1 at both ends (Sec. 2.1, MPS equation).  All routines are plain FP64
numpy; they favour being checkable by eye over speed.
"""
from __future__ import annotations

import numpy as np

from .fermion import C, I2, Z

CUTOFF = 1e-14  # relative singular-value cutoff (reading A5)


def copy(psi):
    return [a.copy() for a in psi]


def bonds(psi):
    return [psi[0].shape[0]] + [a.shape[2] for a in psi]


def scale(psi, c: float):
    """c * |psi>, carried by the last site (norm lives there, reading A5)."""
    out = copy(psi)
    out[-1] = out[-1] * c
    return out


def to_dense(psi) -> np.ndarray:
    """Contract an MPS into the 2^n vector, site 0 most significant."""
    v = psi[0].reshape(psi[0].shape[0] * 2, psi[0].shape[2])
    for a in psi[1:]:
        v = v @ a.reshape(a.shape[0], -1)
        v = v.reshape(-1, a.shape[2])
    return v.reshape(-1)


def overlap(a, b) -> float:
    """<a|b> by the left transfer-matrix chain E_j = sum_n A^nT E_{j-1} B^n."""
    E = np.ones((1, 1))
    for x, y in zip(a, b):
        # E'_cd = sum_{a,n,b} E_ab x_anc y_bnd, contracted in two steps
        F = np.einsum("ab,anc->bnc", E, x)
        E = np.einsum("bnc,bnd->cd", F, y)
    return float(E[0, 0])


def norm(a) -> float:
    return float(np.sqrt(max(overlap(a, a), 0.0)))


# ---------------------------------------------------------------------------
# Elementary bond-2 MPO layer (eq. elementary_MPO) in Jordan-Wigner form.
# W_j = [[Z, y_j o], [0, I]] with o = c (annihilation) or c^T (creation); the
# first site keeps row 0, the last site keeps column 1 (reading A3).
# ---------------------------------------------------------------------------

def layer_mpo(y: np.ndarray, dag: bool):
    """Site tensors W_j[alpha, beta, m, n] of sum_j y_j a_j (or a+_j)."""
    n = y.shape[0]
    o = C.T if dag else C
    ws = []
    for j in range(n):
        w = np.zeros((2, 2, 2, 2))
        w[0, 0] = Z
        w[0, 1] = y[j] * o
        w[1, 1] = I2
        if j == 0:
            w = w[0:1]
        if j == n - 1:
            w = w[:, 1:2]
        ws.append(w)
    return ws


def mpo_to_dense(ws) -> np.ndarray:
    """Contract an MPO into a 2^n x 2^n matrix (the check quoted in Sec. 3.1)."""
    cur = ws[0][0]  # (beta, rows, cols)
    for w in ws[1:]:
        # cur[b, R, C] ; w[b, c, m, n] -> new[c, (R m), (C n)]
        new = np.einsum("bRC,bcmn->cRmCn", cur, w)
        c, R, m, Cc, nn = new.shape
        cur = new.reshape(c, R * m, Cc * nn)
    return cur[0]


def apply_layer(psi, y: np.ndarray, dag: bool):
    """Contract the layer MPO with the MPS on the physical leg (Sec. 2.1):
    B_j[(alpha,a), m, (beta,b)] = sum_n W_j[alpha,beta,m,n] A_j[a,n,b]."""
    ws = layer_mpo(y, dag)
    out = []
    for w, a in zip(ws, psi):
        b = np.einsum("xymn,anb->xamyb", w, a)
        x_, l_, m_, y_, r_ = b.shape
        out.append(b.reshape(x_ * l_, m_, y_ * r_))
    return out


# ---------------------------------------------------------------------------
# Compression (Fig. 3 caption): right-canonical form by QR from the right,
# then SVDs from left to right discarding the smallest singular values and
# merging S V^T into the next site.
# ---------------------------------------------------------------------------

def right_canonicalize(psi):
    """QR sweep right -> left; returns the MPS with sites 1..n-1 right-orthonormal."""
    out = copy(psi)
    for j in range(len(out) - 1, 0, -1):
        a = out[j]
        l, d, r = a.shape
        q, rr = np.linalg.qr(a.reshape(l, d * r).T)  # X^T = Q R  <=>  X = R^T Q^T
        k = q.shape[1]
        out[j] = q.T.reshape(k, d, r)
        out[j - 1] = np.einsum("anb,bk->ank", out[j - 1], rr.T)
    return out


def thin_svd(a: np.ndarray):
    """Thin SVD a = u diag(s) vt, s descending.  LAPACK's divide-and-conquer
    driver (numpy) first; when it reports non-convergence, which it can on
    strongly rank-deficient matrices, the QR-iteration driver (gesvd)."""
    try:
        return np.linalg.svd(a, full_matrices=False)
    except np.linalg.LinAlgError:
        import scipy.linalg
        return scipy.linalg.svd(a, full_matrices=False, lapack_driver="gesvd")


def truncation_rank(s: np.ndarray, D: int, eps: float = CUTOFF) -> int:
    """k = max(1, min(D, #{s_i > eps * s_1})) (reading A5)."""
    if s.size == 0 or s[0] <= 0.0:
        return 1
    return int(max(1, min(D, int(np.count_nonzero(s > eps * s[0])))))


def svd_sweep(psi, D: int, eps: float = CUTOFF, record=None):
    """Left -> right SVD truncation on a right-canonical MPS."""
    out = copy(psi)
    for j in range(len(out) - 1):
        a = out[j]
        l, d, r = a.shape
        u, s, vt = thin_svd(a.reshape(l * d, r))
        k = truncation_rank(s, D, eps)
        if record is not None:
            record.append(s.copy())
        out[j] = u[:, :k].reshape(l, d, k)
        sv = s[:k, None] * vt[:k]
        nxt = out[j + 1]
        out[j + 1] = np.einsum("kb,bnc->knc", sv, nxt)
    return out


def compress(psi, D: int, eps: float = CUTOFF, record=None):
    """QR sweep then SVD sweep; never renormalises (reading A5)."""
    return svd_sweep(right_canonicalize(psi), D, eps, record)


def direct_sum(terms):
    """sum_i c_i |psi_i> as one MPS of bond sum_i chi_i (Sec. 3.2, Alg. 1 addition).

    terms: list of (coefficient, mps).  The coefficient is put on the first
    site; the first site is concatenated along its right bond, interior sites
    are block-diagonal, the last site is concatenated along its left bond.
    """
    n = len(terms[0][1])
    if n == 1:
        return [sum(c * m[0] for c, m in terms)]
    out = []
    for j in range(n):
        blocks = [m[j] for _, m in terms]
        if j == 0:
            out.append(np.concatenate([c * m[0] for c, m in terms], axis=2))
        elif j == n - 1:
            out.append(np.concatenate(blocks, axis=0))
        else:
            L = sum(b.shape[0] for b in blocks)
            R = sum(b.shape[2] for b in blocks)
            t = np.zeros((L, 2, R))
            lo = ro = 0
            for b in blocks:
                t[lo:lo + b.shape[0], :, ro:ro + b.shape[2]] = b
                lo += b.shape[0]
                ro += b.shape[2]
            out.append(t)
    return out


def left_canonical_error(psi) -> float:
    """max_j || sum_n A_j^nT A_j^n - I || over sites 0..n-2."""
    err = 0.0
    for a in psi[:-1]:
        l, d, r = a.shape
        m = a.reshape(l * d, r)
        err = max(err, float(np.max(np.abs(m.T @ m - np.eye(r)))))
    return err


def right_canonical_error(psi) -> float:
    """max_j || sum_n A_j^n A_j^nT - I || over sites 1..n-1."""
    err = 0.0
    for a in psi[1:]:
        l, d, r = a.shape
        m = a.reshape(l, d * r)
        err = max(err, float(np.max(np.abs(m @ m.T - np.eye(l)))))
    return err


def schmidt_values(psi):
    """Schmidt values at every bond (exact, via right-canonical form + SVD sweep)."""
    rec = []
    svd_sweep(right_canonicalize(psi), D=10 ** 9, eps=0.0, record=rec)
    return rec
