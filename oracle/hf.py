"""Closed-form energy of an occupation-number state under eq. (1).

For a determinant with occupations n_{p s} in {0, 1}, taking the operator
order of eq. (1) literally (reading A4):
  <a+_{ps} a_{qs}> = delta_pq n_ps;
  <a+_{ps} a_{qs} a+_{rs'} a_{ss'}> = n_ps n_rs'           (q = p, s = r)
                                    + n_ps (1 - n_qs)       (q = r, s = p, s = s', p != q).
Hence E = sum t_pp n_ps + 1/2 sum v_pprr n_ps n_rs'
          + 1/2 sum_s sum_{p != q} v_pqqp n_ps (1 - n_qs).
"""
from __future__ import annotations

import numpy as np


def determinant_energy(t: np.ndarray, v: np.ndarray, occ) -> float:
    L = t.shape[0]
    n = np.asarray(occ, dtype=float).reshape(L, 2)  # [p, s]
    e = 0.0
    for p in range(L):
        for s in (0, 1):
            e += t[p, p] * n[p, s]
    for p in range(L):
        for s in (0, 1):
            for r in range(L):
                for s2 in (0, 1):
                    e += 0.5 * v[p, p, r, r] * n[p, s] * n[r, s2]
    for s in (0, 1):
        for p in range(L):
            for q in range(L):
                if p != q:
                    e += 0.5 * v[p, q, q, p] * n[p, s] * (1.0 - n[q, s])
    return float(e)


def closed_shell_energy(t: np.ndarray, v: np.ndarray, occupied) -> float:
    """E = 2 sum_{p in O} t_pp + 2 sum_{p,r in O} v_pprr + sum_{p in O, q not in O} v_pqqp."""
    L = t.shape[0]
    O = list(occupied)
    V = [q for q in range(L) if q not in O]
    e = 2.0 * sum(t[p, p] for p in O)
    e += 2.0 * sum(v[p, p, r, r] for p in O for r in O)
    e += sum(v[p, q, q, p] for p in O for q in V)
    return float(e)
