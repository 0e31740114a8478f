"""Krylov time evolution of an MPS (Sec. 2.2, eq. Krylov_combination and the
step a(delta) = exp(-i delta H~) a(0); error bounds of App. A; the NH3 run of
Sec. 4 uses the same scheme).

The molecular H of eq. (1) is real symmetric, so the real and imaginary parts
of a state evolve under real operators.  The state psi = re + i im is held as
a pair of real MPS (reading R10), either of which may be absent (None = the
zero MPS):

* complex overlap  <a|b> = <a_r|b_r> + <a_i|b_i> + i (<a_r|b_i> - <a_i|b_r>);
* compressed H|psi> = (C(H re), C(H im)), one H application per present part;
* compressed sum_j c_j x_j with complex c_j: the real part sums the terms
  (Re c_j, x_j,re), (-Im c_j, x_j,im) for j = 0, 1, ... in that order, the
  imaginary part (Re c_j, x_j,im), (Im c_j, x_j,re); a term whose part is
  absent or whose coefficient is exactly zero is left out, and a part with no
  term left is absent.  Each part is one pairwise-tree sum-compression.

One time step (Sec. 2.2): v_0 = psi / ||psi||; for i = 0 .. K-1:
w_i = C(H v_i), M_ji = <v_j|w_i> (j <= i); unless i = K-1,
r = C(w_i - sum_j M_ji v_j), beta = ||r||, v_{i+1} = r / beta with
S_{i+1,j} = <v_{i+1}|v_j> and M_{i+1,l} = <v_{i+1}|w_l>.  If beta is at or
below BREAKDOWN times sqrt(sum_j |M_ji|^2 + beta^2) (the norm of w_i in an
orthonormal basis) the Krylov space is invariant and the basis stops at
m = i + 1 vectors.  The effective Hamiltonian of eq. eff_H in the
re-orthogonalised basis psi_a = sum_i X_ia v_i (X^H S X = I: Cholesky of S
when every eigenvalue of S exceeds S_EIG_FLOOR, canonical orthogonalisation
otherwise, reading A12) gives a~(delta) = exp(-i delta H~) a~(0) with
a~(0) = X^H S e_0, and psi(t + delta) = ||psi|| sum_i (X a~(delta))_i v_i.
"""
from __future__ import annotations

import numpy as np

from . import mps as M
from .hamiltonian import apply_H, sum_compress
from .lanczos import S_EIG_FLOOR

BREAKDOWN = 1e-10


# ---------------------------------------------------------------------------
# complex states as (re, im) pairs of real MPS (None = zero part)
# ---------------------------------------------------------------------------

def coverlap(a, b) -> complex:
    """<a|b> of two complex states given as (re, im) pairs."""
    def ov(x, y):
        return 0.0 if x is None or y is None else M.overlap(x, y)
    (ar, ai), (br, bi) = a, b
    return complex(ov(ar, br) + ov(ai, bi), ov(ar, bi) - ov(ai, br))


def cnorm(a) -> float:
    return float(np.sqrt(max(coverlap(a, a).real, 0.0)))


def cscale(a, c: float):
    """Real multiple of a complex state."""
    return tuple(None if x is None else M.scale(x, c) for x in a)


def split_terms(coeffs, vecs):
    """The (coefficient, real MPS) term lists of the real and the imaginary
    part of sum_j c_j x_j, in the order stated in the module docstring."""
    re_terms, im_terms = [], []
    for c, (xr, xi) in zip(coeffs, vecs):
        c = complex(c)
        for lst, coef, part in ((re_terms, c.real, xr), (re_terms, -c.imag, xi),
                                (im_terms, c.real, xi), (im_terms, c.imag, xr)):
            if part is not None and coef != 0.0:
                lst.append((coef, part))
    return re_terms, im_terms


def ccombine(coeffs, vecs, D, eps=M.CUTOFF):
    """Compressed sum_j c_j x_j (complex coefficients, complex states)."""
    out = []
    for terms in split_terms(coeffs, vecs):
        if not terms:
            out.append(None)
        else:
            out.append(sum_compress([c for c, _ in terms], [x for _, x in terms], D, eps))
    return tuple(out)


def capply_H(a, t, chi, zeta, D, eps=M.CUTOFF):
    """Compressed H|a> part by part (H real)."""
    return tuple(None if x is None else apply_H(x, t, chi, zeta, D, eps=eps) for x in a)


# ---------------------------------------------------------------------------
# the small problem: a(delta) over the Krylov basis
# ---------------------------------------------------------------------------

def evolution_coefficients(Mm: np.ndarray, S: np.ndarray, delta: float) -> np.ndarray:
    """Coefficients a(delta) over v_0..v_{m-1} of exp(-i delta H~) applied to
    v_0, with H~ the effective Hamiltonian of eq. eff_H built from
    H_sym = (M + M^H)/2 in the re-orthogonalised basis (eq. reortho)."""
    Hs = 0.5 * (Mm + Mm.conj().T)
    s, U = np.linalg.eigh(S)
    if s.size and s[0] > S_EIG_FLOOR:
        X = np.linalg.inv(np.linalg.cholesky(S)).conj().T   # S = L L^H, X = L^{-H}
    else:
        keep = s > S_EIG_FLOOR
        X = U[:, keep] / np.sqrt(s[keep])
    Ht = X.conj().T @ Hs @ X
    lam, W = np.linalg.eigh(Ht)
    e0 = np.zeros(S.shape[0], dtype=complex)
    e0[0] = 1.0
    a0 = X.conj().T @ S @ e0
    at = W @ (np.exp(-1j * delta * lam) * (W.conj().T @ a0))
    return X @ at


# ---------------------------------------------------------------------------
# one time step and a sequence of them
# ---------------------------------------------------------------------------

def evolve_step(psi, t, chi, zeta, D, K, delta, eps=M.CUTOFF, Hfun=None, info=None):
    """psi(t + delta) from psi(t) (both (re, im) pairs) with a Krylov space of
    at most K vectors.  Hfun (optional) replaces the compressed H application
    of one real MPS (tests use an exact dense H).  info, if a dict, receives
    the basis size m and the matrices."""
    H1 = (lambda x: apply_H(x, t, chi, zeta, D, eps=eps)) if Hfun is None else Hfun
    nrm = cnorm(psi)
    if not nrm > 0.0:
        raise ValueError("state has zero norm")
    v = [cscale(psi, 1.0 / nrm)]
    w = []
    Mm = np.zeros((K, K), dtype=complex)
    S = np.zeros((K, K), dtype=complex)
    S[0, 0] = coverlap(v[0], v[0])
    m = K
    for i in range(K):
        wi = tuple(None if x is None else H1(x) for x in v[i])
        w.append(wi)
        for j in range(i + 1):
            Mm[j, i] = coverlap(v[j], wi)
        if i == K - 1:
            break
        r = ccombine([1.0] + [-Mm[j, i] for j in range(i + 1)], [wi] + v[: i + 1], D, eps)
        b = cnorm(r)
        scale_w = np.sqrt(sum(abs(Mm[j, i]) ** 2 for j in range(i + 1)) + b * b)
        if not b > BREAKDOWN * scale_w:
            m = i + 1
            break
        vn = cscale(r, 1.0 / b)
        v.append(vn)
        for j in range(i + 2):
            S[i + 1, j] = coverlap(vn, v[j])
            S[j, i + 1] = np.conj(S[i + 1, j])
        for l in range(i + 1):
            Mm[i + 1, l] = coverlap(vn, w[l])
    a = nrm * evolution_coefficients(Mm[:m, :m], S[:m, :m], delta)
    if info is not None:
        info.update(m=m, M=Mm[:m, :m].copy(), S=S[:m, :m].copy(), a=a.copy())
    return ccombine(list(a), v[:m], D, eps)


def evolve(psi, t, chi, zeta, D, K, delta, n_steps, eps=M.CUTOFF, Hfun=None):
    """n_steps Krylov time steps; returns the final (re, im) pair and the
    basis size of every step."""
    dims = []
    for _ in range(n_steps):
        info = {}
        psi = evolve_step(psi, t, chi, zeta, D, K, delta, eps, Hfun, info)
        dims.append(info["m"])
    return psi, dims


def to_dense_complex(a) -> np.ndarray:
    """Dense 2^n complex vector of an (re, im) pair."""
    re, im = a
    ref = re if re is not None else im
    n = 2 ** len(ref)
    vr = M.to_dense(re) if re is not None else np.zeros(n)
    vi = M.to_dense(im) if im is not None else np.zeros(n)
    return vr + 1j * vi
