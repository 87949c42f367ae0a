"""Damped Roothaan self-consistent field loop for the model functional (test
infrastructure only).

The paper compares ETDM with the SCF method (Sec. 3.5, Sec. 4); here the SCF
fixed point serves as an independent check of where the minimum lies: at
self-consistency the occupied orbitals are the lowest eigenvectors of
H(rho) = H0 + U diag(rho_mu_mu), a stationary point of E that L-BFGS must reach
from A = 0 when both converge.
"""
from __future__ import annotations

import numpy as np


def scf_minimum(H0: np.ndarray, N: int, f_occ: float, hubbard_U: float, rho0: np.ndarray,
                mix: float = 0.3, tol: float = 1e-13, max_iter: int = 2000):
    rho = rho0.copy()
    for it in range(max_iter):
        n = np.real(np.diag(rho))
        H = H0 + hubbard_U * np.diag(n)
        _, C = np.linalg.eigh(H)
        Co = C[:, :N]
        rho_new = f_occ * Co @ Co.conj().T
        diff = np.abs(rho_new - rho).max()
        if diff < tol:
            n = np.real(np.diag(rho_new))
            E = float(np.real(np.trace(rho_new @ H0))) + 0.5 * hubbard_U * float((n ** 2).sum())
            return E, rho_new, it
        rho = (1.0 - mix) * rho + mix * rho_new
    raise RuntimeError("SCF did not converge")
