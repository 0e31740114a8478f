"""Jordan-Wigner fermions and dense Fock-space Hamiltonians (oracle).

Conventions (App. C, readings A1/A2):
* n = 2L spin-orbital sites, site j = 2p + s (s = 0 up, s = 1 down), so the
  up orbital precedes the down orbital of the same spatial orbital, as in
  App. C where b_up = c (x) I and b_down = Z (x) c.
* local basis (|empty>, |occupied>); c = [[0, 1], [0, 0]] (App. C);
  Z = diag(1, -1); a_j = Z_0 ... Z_{j-1} c_j (Sec. 3.1, JW substitution).
* dense index = sum_j n_j 2^(n-1-j): site 0 is the most significant bit,
  i.e. numpy kron order op_0 (x) op_1 (x) ... .
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

C = np.array([[0.0, 1.0], [0.0, 0.0]])
Z = np.diag([1.0, -1.0])
I2 = np.eye(2)


def jw_annihilator(j: int, n: int) -> sp.csr_matrix:
    """Sparse a_j = Z^{(x)j} (x) c (x) I^{(x)(n-j-1)} on 2^n states."""
    out = sp.identity(1, format="csr")
    for k in range(n):
        if k < j:
            op = Z
        elif k == j:
            op = C
        else:
            op = I2
        out = sp.kron(out, sp.csr_matrix(op), format="csr")
    return out


def annihilators(n: int) -> list:
    return [jw_annihilator(j, n) for j in range(n)]


def hamiltonian_sparse(t: np.ndarray, v: np.ndarray) -> sp.csr_matrix:
    """H of eq. (1), operator order exactly as printed (reading A4).

    H = sum_{pq,s} t_pq a+_{ps} a_{qs}
      + 1/2 sum_{pqrs,s,s'} v_pqrs a+_{ps} a_{qs} a+_{rs'} a_{ss'}.
    With E_pq = sum_s a+_{ps} a_{qs} this is sum t_pq E_pq
    + 1/2 sum v_pqrs E_pq E_rs.
    """
    L = t.shape[0]
    n = 2 * L
    a = annihilators(n)
    E = {}
    for p in range(L):
        for q in range(L):
            E[p, q] = a[2 * p].T @ a[2 * q] + a[2 * p + 1].T @ a[2 * q + 1]
    H = sp.csr_matrix((2 ** n, 2 ** n))
    for p in range(L):
        for q in range(L):
            if t[p, q] != 0.0:
                H = H + t[p, q] * E[p, q]
    for p in range(L):
        for q in range(L):
            for r in range(L):
                for s in range(L):
                    if v[p, q, r, s] != 0.0:
                        H = H + 0.5 * v[p, q, r, s] * (E[p, q] @ E[r, s])
    return H.tocsr()


# ---- dense-vector operator application (no matrices; any n up to ~24) ----

def _prefix_parity_sign(j: int) -> np.ndarray:
    """(-1)^(number of occupied sites among 0..j-1) for each prefix index."""
    idx = np.arange(2 ** j, dtype=np.int64)
    pop = np.zeros_like(idx)
    x = idx.copy()
    while np.any(x):
        pop += x & 1
        x >>= 1
    return np.where(pop % 2 == 0, 1.0, -1.0)


def apply_a(vec: np.ndarray, j: int, n: int, dag: bool = False) -> np.ndarray:
    """a_j |vec> (or a+_j) for a dense vector in the site-0-major basis."""
    x = vec.reshape(2 ** j, 2, 2 ** (n - j - 1))
    out = np.zeros_like(x)
    if dag:
        out[:, 1, :] = x[:, 0, :]
    else:
        out[:, 0, :] = x[:, 1, :]
    out *= _prefix_parity_sign(j)[:, None, None]
    return out.reshape(-1)


def apply_E(vec: np.ndarray, p: int, q: int, L: int) -> np.ndarray:
    """E_pq |vec> = sum_s a+_{ps} a_{qs} |vec>."""
    n = 2 * L
    out = np.zeros_like(vec)
    for s in (0, 1):
        out += apply_a(apply_a(vec, 2 * q + s, n), 2 * p + s, n, dag=True)
    return out


def apply_H_dense(vec: np.ndarray, t: np.ndarray, v: np.ndarray) -> np.ndarray:
    """H|vec> with H from eq. (1) written out on a dense vector.

    T|vec> = sum_pq t_pq E_pq |vec>;  V|vec> = 1/2 sum_pq E_pq w_pq with
    w_pq = sum_rs v_pqrs E_rs |vec>.  This is the plain definition, only
    regrouped by the associativity of the sums.
    """
    L = t.shape[0]
    phi = np.stack([apply_E(vec, r, s, L) for r in range(L) for s in range(L)])
    out = (t.reshape(-1) @ phi)
    w = v.reshape(L * L, L * L) @ phi
    k = 0
    for p in range(L):
        for q in range(L):
            out = out + 0.5 * apply_E(w[k], p, q, L)
            k += 1
    return out


def number_operator_dense(n: int) -> np.ndarray:
    """Diagonal of the total particle number on 2^n states."""
    idx = np.arange(2 ** n, dtype=np.int64)
    pop = np.zeros_like(idx)
    for j in range(n):
        pop += (idx >> (n - 1 - j)) & 1
    return pop.astype(float)


def sz_dense(n: int) -> np.ndarray:
    """Diagonal of 2*S_z = N_up - N_down on 2^n states (site j = 2p + s)."""
    idx = np.arange(2 ** n, dtype=np.int64)
    out = np.zeros(2 ** n)
    for j in range(n):
        bit = (idx >> (n - 1 - j)) & 1
        out += bit if j % 2 == 0 else -bit
    return out
