"""THC factors, spin-site coefficient vectors and the kinetic split (oracle)."""
from __future__ import annotations

import numpy as np


def thc_v(chi: np.ndarray, zeta: np.ndarray) -> np.ndarray:
    """v_pqrs = sum_{mu nu} chi_p^mu chi_q^mu zeta^{mu nu} chi_r^nu chi_s^nu (eq. thc)."""
    return np.einsum("pm,qm,mn,rn,sn->pqrs", chi, chi, zeta, chi, chi)


def spin_site_coeffs(x: np.ndarray, sigma: int) -> np.ndarray:
    """Coefficients of sum_p x_p a_{p sigma} on the 2L spin-orbital sites.

    y_j = x_p when j = 2p + sigma, else 0 (site layout reading A1).
    """
    L = x.shape[0]
    y = np.zeros(2 * L)
    y[sigma::2] = x
    return y


def kinetic_split(t: np.ndarray):
    """t = u diag(lam) u^T (App. D, eq. t_diagonalization); lam ascending."""
    lam, u = np.linalg.eigh(t)
    return lam, u


def v_terms(N: int):
    """V-term order of Algorithm 1 (reading A10): nu outer, sigma' inner,
    then mu, sigma; spins ordered (up, down)."""
    for nu in range(N):
        for sp_ in (0, 1):
            for mu in range(N):
                for s in (0, 1):
                    yield nu, sp_, mu, s
