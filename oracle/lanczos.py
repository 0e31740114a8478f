"""Global Krylov (Lanczos) step on MPS (Sec. 2.2; readings A12, A13).

Step i, given orthonormalised Krylov MPS v_0..v_i:
  w_i = compressed H|v_i>                       (Sec. 3.2 / Algorithm 1)
  h_ji = <v_j|w_i> for j <= i                   (eq. Krylov_H)
  r = compress(w_i - sum_j h_ji v_j)             (Gram-Schmidt w.r.t. all previous)
  beta_i = ||r||,  v_{i+1} = r / beta_i
  S_{i+1,j} = <v_{i+1}|v_j>,  M_{i+1,l} = <v_{i+1}|w_l>
Ritz values: (1) the tridiagonal (alpha_i = h_ii, beta_i) the paper assumes;
(2) the generalised problem (H_sym, S) with H_sym = (M + M^T)/2, solved in
the re-orthogonalised basis psi_a = sum_i C_ai v_i with C S C^T = I
(eq. reortho, eq. eff_H): Cholesky, or canonical orthogonalisation when S is
numerically singular.
"""
from __future__ import annotations

import numpy as np

from . import mps as M
from .hamiltonian import apply_H, sum_compress

S_EIG_FLOOR = 1e-10


def ritz_tridiagonal(alpha, beta):
    """Eigenvalues of the Lanczos tridiagonal: alpha_i on the diagonal,
    beta_i between basis vectors i and i+1 (Sec. 2.2)."""
    m = len(alpha)
    T = np.diag(np.asarray(alpha, float))
    for k in range(m - 1):
        T[k, k + 1] = T[k + 1, k] = beta[k]
    return np.linalg.eigvalsh(T)


def ritz_generalized(Hm: np.ndarray, S: np.ndarray):
    """Eigenvalues of H_sym = (M + M^T)/2 in the re-orthogonalised basis
    psi_a = sum_i C_ai v_i with C S C^T = I (eq. reortho, eq. eff_H).

    When every eigenvalue of S exceeds S_EIG_FLOOR, C = L^{-1} with S = L L^T
    (Cholesky) and all m values are returned.  Otherwise S is numerically
    singular and the basis is canonically orthogonalised: C = s^{-1/2} U^T
    over the eigenpairs (s, U) of S with s > S_EIG_FLOOR, giving fewer
    values (reading A12).
    """
    Hs = 0.5 * (Hm + Hm.T)
    s, U = np.linalg.eigh(S)
    if s.size and s[0] > S_EIG_FLOOR:
        Cm = np.linalg.inv(np.linalg.cholesky(S))
        return np.linalg.eigvalsh(Cm @ Hs @ Cm.T)
    keep = s > S_EIG_FLOOR
    X = U[:, keep] / np.sqrt(s[keep])
    return np.linalg.eigvalsh(X.T @ Hs @ X)


def ritz_pairs(Hm: np.ndarray, S: np.ndarray):
    """Ritz values w_a and coefficient vectors X[:, a] of the generalised
    problem of ``ritz_generalized``: psi_a = sum_i X[i, a] v_i is the Ritz
    vector of w_a, normalised in the metric S (X^T S X = I).  With C the
    re-orthogonalising transform (rows c_b) and y_a the eigenvectors of
    C H_sym C^T, X = C^T Y (eq. reortho, eq. eff_H)."""
    Hs = 0.5 * (Hm + Hm.T)
    s, U = np.linalg.eigh(S)
    if s.size and s[0] > S_EIG_FLOOR:
        Cm = np.linalg.inv(np.linalg.cholesky(S))
    else:
        keep = s > S_EIG_FLOOR
        Cm = (U[:, keep] / np.sqrt(s[keep])).T
    w, Y = np.linalg.eigh(Cm @ Hs @ Cm.T)
    return w, Cm.T @ Y


class KrylovState:
    def __init__(self, v0, K: int):
        nv = M.norm(v0)
        self.v = [M.scale(v0, 1.0 / nv)]
        self.w = []
        self.K = K
        self.Mm = np.zeros((K + 1, K + 1))
        self.S = np.zeros((K + 1, K + 1))
        self.S[0, 0] = M.overlap(self.v[0], self.v[0])
        self.alpha = []
        self.beta = []
        self.breakdown = False

    @property
    def i(self):
        return len(self.w)


def krylov_step(st: KrylovState, t, chi, zeta, D, mode="tree", eps=M.CUTOFF, Hfun=None):
    """One Lanczos step; returns (ritz_generalized, ritz_tridiagonal, beta_i)."""
    i = st.i
    vi = st.v[i]
    wi = apply_H(vi, t, chi, zeta, D, mode=mode, eps=eps) if Hfun is None else Hfun(vi)
    st.w.append(wi)
    for j in range(i + 1):
        st.Mm[j, i] = M.overlap(st.v[j], wi)
    st.alpha.append(st.Mm[i, i])
    coeffs = [1.0] + [-st.Mm[j, i] for j in range(i + 1)]
    r = sum_compress(coeffs, [wi] + st.v[: i + 1], D, eps)
    b = M.norm(r)
    st.beta.append(b)
    if b > 0.0 and i + 1 <= st.K:
        v_new = M.scale(r, 1.0 / b)
        st.v.append(v_new)
        for j in range(i + 2):
            st.S[i + 1, j] = st.S[j, i + 1] = M.overlap(v_new, st.v[j])
        for l in range(i + 1):
            st.Mm[i + 1, l] = M.overlap(v_new, st.w[l])
    else:
        st.breakdown = True
    m = i + 1
    rg = ritz_generalized(st.Mm[:m, :m], st.S[:m, :m])
    rt = ritz_tridiagonal(st.alpha[:m], st.beta[: m - 1])
    return rg, rt, b


def dense_lanczos(Hmat_apply, v0: np.ndarray, K: int):
    """Textbook Lanczos with full Gram-Schmidt on dense vectors (pin reference)."""
    v = [v0 / np.linalg.norm(v0)]
    Hv = []
    ritz = []
    for i in range(K):
        w = Hmat_apply(v[i])
        Hv.append(w)
        r = w - sum((vj @ w) * vj for vj in v)
        m = i + 1
        Vm = np.stack(v)
        Hp = Vm @ np.stack(Hv).T
        ritz.append(np.linalg.eigvalsh(0.5 * (Hp + Hp.T)))
        b = np.linalg.norm(r)
        if b < 1e-12:
            break
        v.append(r / b)
    return ritz


def ritz_vector(st: KrylovState, a: int, D: int, eps=M.CUTOFF):
    """MPS of the a-th Ritz vector (ascending Ritz values) over the basis
    v_0..v_{m-1} of the steps taken: sum_i X[i, a] v_i, summed by
    ``sum_compress`` (Sec. 2.2, eq. reortho)."""
    m = st.i
    _, X = ritz_pairs(st.Mm[:m, :m], st.S[:m, :m])
    return sum_compress(list(X[:, a]), st.v[:m], D, eps)


def restart(st: KrylovState, a: int, D: int, K: int = None, eps=M.CUTOFF) -> KrylovState:
    """A new Krylov state started from the a-th Ritz vector of st (the
    restart the paper uses to recover convergence lost to truncation,
    Sec. 2.2); the new start vector is normalised by KrylovState."""
    return KrylovState(ritz_vector(st, a, D, eps), st.K if K is None else K)


def dense_lanczos_restarted(Hmat_apply, v0: np.ndarray, K: int, restarts: int, a: int = 0):
    """Textbook dense Lanczos (full Gram-Schmidt) restarted ``restarts`` times
    from its a-th Ritz vector after every K steps (pin reference).  Returns
    the Ritz values after every step."""
    out = []
    v0 = v0 / np.linalg.norm(v0)
    for _ in range(restarts + 1):
        V = [v0]
        for i in range(K):
            w = Hmat_apply(V[i])
            Vm = np.stack(V)
            Hp = Vm @ np.stack([Hmat_apply(x) for x in V]).T
            vals, vecs = np.linalg.eigh(0.5 * (Hp + Hp.T))
            out.append(vals)
            r = w - sum((x @ w) * x for x in V)
            r = r - sum((x @ r) * x for x in V)
            b = np.linalg.norm(r)
            if i + 1 < K and b > 1e-12:
                V.append(r / b)
            else:
                break
        v0 = np.stack(V).T @ vecs[:, a]
        v0 = v0 / np.linalg.norm(v0)
    return out
