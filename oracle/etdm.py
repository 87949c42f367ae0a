"""FP64 reference implementation of E(A) and dE/dA for exponential-transformation
direct minimization (test infrastructure only; see the package docstring).

Notation (the paper's, with one renaming):
  A       skew-Hermitian generator, one per instance / k-point (Sec. 2, Eq. unit_transf)
  U       = exp(A), the unitary of Eq. unit_transf
  V, w    eigenvectors / eigenvalues of iA (the paper calls the eigenvectors U in
          Eq. ed; renamed here to keep U = exp(A))
  C0      reference orbitals, C = C0 exp(A) are the current orbitals (the paper's O)
  F       diag(f), occupation numbers
  rho     density matrix rho = C F C^dagger (Sec. 2, definition of rho_mu_nu)
  H       Hamiltonian matrix dE/drho^T (Sec. 2, Eq. der_of_en_1)
  H_MO    C^dagger H C, L = [F, H_MO] (Sec. 2, definition of L_mk)
  Y       integral_0^1 exp(tA) L exp(-tA) dt  (Sec. 2, Eq. gradients)

Model energy functional (replaces the Kohn-Sham functional, which needs grids):
  E = sum_k w_k Tr(rho_k H0_k) + (U_hub / 2) sum_mu n_mu^2
  n_mu = rho_mu_mu of each instance (independent instances), or the
  weight-averaged sum_k w_k (rho_k)_mu_mu when the instances are k-points of one
  crystal ("couple").  Then H_k = H0_k + U_hub diag(n), which is Hermitian and
  unitary invariant, as Eq. der_of_en_1 requires.
"""
from __future__ import annotations

from typing import List, Sequence, Tuple

import numpy as np
import scipy.linalg

# ----------------------------------------------------------------------------
# parameters <-> generator A
# ----------------------------------------------------------------------------


def ov_generator(B: np.ndarray) -> np.ndarray:
    """Hutter's occupied-virtual parametrization A = [[0, B], [-B^dagger, 0]] (Sec. 3.4)."""
    N, Nv = B.shape
    A = np.zeros((N + Nv, N + Nv), dtype=B.dtype)
    A[:N, N:] = B
    A[N:, :N] = -B.conj().T
    return A


def skew_from_upper(a: np.ndarray) -> np.ndarray:
    """Skew-Hermitian A from its upper triangle incl. the diagonal (Sec. 2: E is a
    function of the upper-triangular elements; Re of the diagonal is zero)."""
    up = np.triu(a, 1)
    d = 1j * np.imag(np.diag(a)) if np.iscomplexobj(a) else np.zeros(a.shape[0])
    return up - up.conj().T + np.diag(d)


def generator(kind: str, a: np.ndarray) -> np.ndarray:
    if kind == "real_ov":
        return ov_generator(a)
    if kind == "complex_full":
        return skew_from_upper(a)
    raise ValueError(kind)


# ----------------------------------------------------------------------------
# matrix exponential
# ----------------------------------------------------------------------------


def eig_iA(A: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """Eigendecomposition iA = V diag(w) V^dagger of the Hermitian matrix iA (Sec. 3.4)."""
    w, V = np.linalg.eigh(1j * A)
    return w, V


def expm_eig(A: np.ndarray) -> np.ndarray:
    """exp(A) = V exp(-i w) V^dagger from the eigendecomposition of iA (Eq. ed)."""
    w, V = eig_iA(A)
    U = (V * np.exp(-1j * w)[None, :]) @ V.conj().T
    return U.real.copy() if np.isrealobj(A) else U


def expm_pade(A: np.ndarray) -> np.ndarray:
    """Scaling and squaring with Pade approximant (Eq. ss; SciPy's Al-Mohy-Higham),
    an independent algorithm used to cross-check expm_eig and expm_ss."""
    return scipy.linalg.expm(A)


# Eq. ss: exp(A) = exp(A / 2^s)^(2^s) with the [m/m] Pade approximant of exp(A / 2^s).
# theta_m: the largest 1-norm of the scaled matrix for which the [m/m] approximant has
# backward error below the FP64 unit roundoff (the table of Higham's scaling and
# squaring method, which the Al-Mohy-Higham algorithm refines).
PADE_THETA = ((3, 1.495585217958292e-2), (5, 2.539398330063230e-1), (7, 9.504178996162932e-1),
              (9, 2.097847961257068e0), (13, 5.371920351148152e0))


def pade_coefficients(m: int) -> List[float]:
    """Numerator coefficients b_j of the [m/m] Pade approximant of exp: p(x) = sum_j b_j x^j,
    b_j = (2m - j)! m! / ((2m)! j! (m - j)!), and the denominator is q(x) = p(-x)."""
    from math import factorial
    return [factorial(2 * m - j) * factorial(m) / (factorial(2 * m) * factorial(j) * factorial(m - j))
            for j in range(m + 1)]


def pade_degree_and_scaling(norm1: float) -> Tuple[int, int]:
    """(m, s): the smallest tabulated m whose theta_m covers the 1-norm; beyond theta_13,
    m = 13 and the fewest halvings s that bring the norm under theta_13."""
    for m, theta in PADE_THETA[:-1]:
        if norm1 <= theta:
            return m, 0
    theta13 = PADE_THETA[-1][1]
    s = 0
    while norm1 / 2.0 ** s > theta13:
        s += 1
    return 13, s


def expm_ss(A: np.ndarray) -> np.ndarray:
    """exp(A) by scaling and squaring with a diagonal Pade approximant (Eq. ss): scale by
    2^-s, evaluate q(X)^-1 p(X) from plain powers of X, square s times."""
    m, s = pade_degree_and_scaling(float(np.abs(A).sum(axis=0).max()))
    X = A / 2.0 ** s
    b = pade_coefficients(m)
    P = np.zeros_like(X)
    Q = np.zeros_like(X)
    Xj = np.eye(A.shape[0], dtype=X.dtype)
    for j in range(m + 1):
        P = P + b[j] * Xj
        Q = Q + (-1.0) ** j * b[j] * Xj
        Xj = Xj @ X
    R = np.linalg.solve(Q, P)
    for _ in range(s):
        R = R @ R
    return R


def frechet_expm_ss(A: np.ndarray, E: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """exp(A) and its Frechet derivative L(A, E) = d/dh exp(A + h E) at h = 0 by scaling and
    squaring (Eq. ss differentiated): with X = A / 2^s and r = q(X)^-1 p(X), the derivative of
    every power X^j follows the product rule, L_r = q^-1 (L_p - L_q r), and each squaring
    R <- R R carries L <- R L + L R."""
    m, s = pade_degree_and_scaling(float(np.abs(A).sum(axis=0).max()))
    X, Es = A / 2.0 ** s, E / 2.0 ** s
    b = pade_coefficients(m)
    n = A.shape[0]
    dt = np.result_type(X, Es)
    P, Q, LP, LQ = (np.zeros((n, n), dtype=dt) for _ in range(4))
    Xj = np.eye(n, dtype=dt)
    Lj = np.zeros((n, n), dtype=dt)  # derivative of X^j
    for j in range(m + 1):
        sign = (-1.0) ** j
        P, Q = P + b[j] * Xj, Q + sign * b[j] * Xj
        LP, LQ = LP + b[j] * Lj, LQ + sign * b[j] * Lj
        Lj = X @ Lj + Es @ Xj
        Xj = Xj @ X
    R = np.linalg.solve(Q, P)
    L = np.linalg.solve(Q, LP - LQ @ R)
    for _ in range(s):
        R, L = R @ R, R @ L + L @ R
    return R, L


def _sinc(x):
    """sin(x)/x with the value 1 at x = 0 (np.sinc is sin(pi x)/(pi x))."""
    return np.sinc(np.asarray(x) / np.pi)


def expm_ov(B: np.ndarray) -> np.ndarray:
    """Closed-form exp(A) for A = [[0, B], [-B^T, 0]] (real B), Eq. uinv.

    Reading of the garbled printed equation: with P = B B^T,
      top-left     cos(P^{1/2})
      top-right    P^{-1/2} sin(P^{1/2}) B
      bottom-left  -B^T P^{-1/2} sin(P^{1/2})
      bottom-right I + B^T (cos(P^{1/2}) - I) P^{-1} B
    Every block is an entire function of P, evaluated through P = X diag(s) X^T.
    """
    N, Nv = B.shape
    s, X = np.linalg.eigh(B @ B.T)
    sig = np.sqrt(np.clip(s, 0.0, None))
    cosP = (X * np.cos(sig)) @ X.T
    sincP = (X * _sinc(sig)) @ X.T
    # (cos(x) - 1)/x^2 = -1/2 sinc(x/2)^2 (entire; no inverse of P needed)
    WP = (X * (-0.5 * _sinc(0.5 * sig) ** 2)) @ X.T
    U = np.empty((N + Nv, N + Nv))
    U[:N, :N] = cosP
    U[:N, N:] = sincP @ B
    U[N:, :N] = -B.T @ sincP
    U[N:, N:] = np.eye(Nv) + B.T @ WP @ B
    return U


# ----------------------------------------------------------------------------
# energy and gradient: the definition (dense eigenbasis of iA)
# ----------------------------------------------------------------------------


def divided_difference_factor(w: np.ndarray) -> np.ndarray:
    """D_pq = integral_0^1 exp(-i t (w_p - w_q)) dt = exp(-i x/2) sinc(x/2), x = w_p - w_q.

    This is the Hadamard factor of the gradient formula in Sec. 3.4, with the sign
    taken from Eq. gradients (the printed (exp(-ix) - 1)/(ix) is its negative).
    """
    x = w[:, None] - w[None, :]
    return np.exp(-0.5j * x) * _sinc(0.5 * x)


def overlap_sqrt(inst):
    """S^(1/2) of a non-orthogonal basis (principal square root through eigh), or None."""
    if inst.S is None:
        return None
    s, V = np.linalg.eigh(inst.S)
    return (V * np.sqrt(s)[None, :]) @ V.conj().T


def _densities(wl, params, expm=None):
    """Current orbitals C = C0 exp(A) and the site populations n_mu: the diagonal of
    rho = C F C^dagger, or in a non-orthogonal basis (C^dagger S C = I, Sec. 2) the Lowdin
    populations, the diagonal of S^(1/2) rho S^(1/2) (reading: the model's site density
    with S != I).  exp(A) by the eigendecomposition of iA unless another is given."""
    expm = expm or expm_eig
    Cs, ds = [], []
    for inst, a in zip(wl.instances, params):
        A = generator(wl.kind, a)
        C = inst.C0 @ expm(A)
        Cs.append(C)
        Sh = overlap_sqrt(inst)
        Cd = C if Sh is None else Sh @ C
        ds.append((np.abs(Cd) ** 2 * inst.f[None, :]).sum(axis=1))
    return Cs, ds


def _hamiltonian(inst, n, hubbard_U):
    """H = dE/drho^T: H0 + U diag(n), or H0 + U S^(1/2) diag(n) S^(1/2) with an overlap."""
    Sh = overlap_sqrt(inst)
    if Sh is None:
        return inst.h0_dense() + hubbard_U * np.diag(n)
    return inst.h0_dense() + hubbard_U * (Sh * n[None, :]) @ Sh


def _hubbard_density(wl, ds):
    if wl.couple:
        n = sum(inst.weight * d for inst, d in zip(wl.instances, ds))
        return [n] * len(ds)
    return list(ds)


def energy(wl, params, expm=None) -> float:
    """Total energy E(A) of the workload (all instances)."""
    Cs, ds = _densities(wl, params, expm)
    ns = _hubbard_density(wl, ds)
    E = 0.0
    for inst, C in zip(wl.instances, Cs):
        H0 = inst.h0_dense()
        E += inst.weight * float(np.real(np.einsum("m,mm->", inst.f, C.conj().T @ H0 @ C)))
    if wl.couple:
        E += 0.5 * wl.hubbard_U * float((ns[0] ** 2).sum())
    else:
        E += 0.5 * wl.hubbard_U * float(sum((n ** 2).sum() for n in ns))
    return E


def energy_grad(wl, params) -> Tuple[float, List[np.ndarray]]:
    """E(A) and the gradient with respect to the free variables, per instance.

    Follows Sec. 2: H = H0 + U diag(n); H_MO = C^dagger H C; L = w [F, H_MO];
    dE/da_ij = (2 - delta_ij)/2 * Y_ji with Y from the eigenbasis of iA (Sec. 3.4);
    dE/dRe a = 2 Re(dE/da), dE/dIm a = -2 Im(dE/da).

    Returned gradients:
      real_ov      g[i, j] = dE/dB_ij, B_ij = a_{i, N+j}  (real N x Nv)
      complex_full G[i, j] = dE/dRe a_ij + i dE/dIm a_ij on i <= j, 0 below
                   (Re of the diagonal is not a variable: G_ii is purely imaginary)
    """
    Cs, ds = _densities(wl, params)
    ns = _hubbard_density(wl, ds)
    E = energy(wl, params)
    grads = []
    for inst, a, C, n in zip(wl.instances, params, Cs, ns):
        A = generator(wl.kind, a)
        H = _hamiltonian(inst, n, wl.hubbard_U)
        H_MO = C.conj().T @ H @ C
        F = np.diag(inst.f)
        L = inst.weight * (F @ H_MO - H_MO @ F)
        w, V = eig_iA(A)
        Lt = V.conj().T @ L @ V
        Y = V @ (Lt * divided_difference_factor(w)) @ V.conj().T
        M = A.shape[0]
        delta = np.eye(M)
        dEda = 0.5 * (2.0 - delta) * Y.T  # dE/da_ij = (2 - delta_ij)/2 Y_ji
        dRe = 2.0 * np.real(dEda)
        dIm = -2.0 * np.imag(dEda)
        if wl.kind == "real_ov":
            N = inst.N
            grads.append(dRe[:N, N:].copy())
        else:
            G = np.triu(dRe, 1) + 1j * np.triu(dIm)
            grads.append(G)
    return E, grads


def energy_grad_approx(wl, params, expm=None, lam: float = 0.0) -> Tuple[float, List[np.ndarray]]:
    """E(A) and the approximate gradient G ~ L^T of Sec. 3.4, Eq. app_grad: the first
    term of the gradient expansion, with L = w [F, H_MO] at the current orbitals
    C = C0 exp(A).  It replaces Y by L in energy_grad (exact at A = 0, where the
    divided-difference factors are all 1); same layout of the returned gradients.
    expm selects the exponential (expm_ss: the scaling-and-squaring configuration).
    lam != 0 adds the orbital-dependent model term (complex kind) to E and its part to L,
    as in energy_grad_odd.
    """
    Cs, ds = _densities(wl, params, expm)
    ns = _hubbard_density(wl, ds)
    E = energy(wl, params, expm) if lam == 0.0 else energy_odd(wl, params, lam, expm)
    grads = []
    for inst, C, n in zip(wl.instances, Cs, ns):
        H = _hamiltonian(inst, n, wl.hubbard_U)
        H_MO = C.conj().T @ H @ C
        F = np.diag(inst.f)
        L = inst.weight * (F @ H_MO - H_MO @ F)
        if lam != 0.0:
            assert wl.kind == "complex_full"
            V = orbital_potential_elements(_lowdin_orbitals(inst, C), lam)
            L = L + inst.weight * (inst.f[:, None] * V.T.conj() - inst.f[None, :] * V)
        M = L.shape[0]
        delta = np.eye(M)
        dEda = 0.5 * (2.0 - delta) * L.T  # G = 2 / (2 - delta) dE/da ~ L^T
        dRe = 2.0 * np.real(dEda)
        dIm = -2.0 * np.imag(dEda)
        if wl.kind == "real_ov":
            N = inst.N
            grads.append(dRe[:N, N:].copy())
        else:
            grads.append(np.triu(dRe, 1) + 1j * np.triu(dIm))
    return E, grads


def energy_grad_ss(wl, params) -> Tuple[float, List[np.ndarray]]:
    """E(A) and the exact gradient with exp(A) and Y from scaling and squaring: since
    exp(A) is unitary, Y = integral_0^1 e^{tA} L e^{-tA} dt = L(A, L) exp(A)^dagger with L(A, .)
    the Frechet derivative of exp (no eigendecomposition).  Same layout as energy_grad."""
    Cs, ds = _densities(wl, params, expm_ss)
    ns = _hubbard_density(wl, ds)
    E = energy(wl, params, expm_ss)
    grads = []
    for inst, a, C, n in zip(wl.instances, params, Cs, ns):
        H = _hamiltonian(inst, n, wl.hubbard_U)
        H_MO = C.conj().T @ H @ C
        F = np.diag(inst.f)
        L = inst.weight * (F @ H_MO - H_MO @ F)
        U, LA = frechet_expm_ss(generator(wl.kind, a), L)
        Y = LA @ U.conj().T
        M = L.shape[0]
        delta = np.eye(M)
        dEda = 0.5 * (2.0 - delta) * Y.T
        dRe = 2.0 * np.real(dEda)
        dIm = -2.0 * np.imag(dEda)
        if wl.kind == "real_ov":
            grads.append(dRe[:inst.N, inst.N:].copy())
        else:
            grads.append(np.triu(dRe, 1) + 1j * np.triu(dIm))
    return E, grads


# ----------------------------------------------------------------------------
# an orbital-dependent term (Sec. 2: the L of a functional that depends on the
# orbitals as well as on the density, the PZ-SIC form)
# ----------------------------------------------------------------------------
#
# Model (stands in for PZ-SIC, whose orbital densities need grids): every orbital k
# interacts with its own site density n^(k)_mu = |C_mu_k|^2 (orthonormal basis),
#   E_odd = -(lam / 2) sum_k w f_k sum_mu |C_mu_k|^4,
# an orbital potential V^k = diag(-lam |C_mu_k|^2), V_mk = <m|V^k|k>.


def orbital_potential_elements(C: np.ndarray, lam: float) -> np.ndarray:
    """V[m, k] = <m|V^k|k> = sum_mu conj(C_mu_m) (-lam |C_mu_k|^2) C_mu_k."""
    v = -lam * np.abs(C) ** 2
    return C.conj().T @ (v * C)


def _lowdin_orbitals(inst, C):
    """The orbitals' coefficients on the orthonormalized sites: S^(1/2) C with an overlap
    (reading: the orbital densities of the model term are Lowdin site densities, as the
    site density of the Hubbard term is), C itself without one."""
    Sh = overlap_sqrt(inst)
    return C if Sh is None else Sh @ C


def energy_odd(wl, params, lam: float, expm=None) -> float:
    """E(A) of energy() plus the orbital-dependent model term."""
    Cs, _ = _densities(wl, params, expm)
    E = energy(wl, params, expm)
    for inst, C in zip(wl.instances, Cs):
        Cl = _lowdin_orbitals(inst, C)
        E += -0.5 * lam * inst.weight * float((inst.f[None, :] * np.abs(Cl) ** 4).sum())
    return E


def energy_grad_odd(wl, params, lam: float, printed_indices: bool = False) -> Tuple[float, List[np.ndarray]]:
    """E and the exact gradient with the orbital-dependent term (complex full
    parametrization; the ov form assumes unitary invariance).  For an energy that
    depends on the orbitals C, with Gamma = dE/dC^* and G = Gamma^dagger C, the L of
    Eq. gradients is G - G^dagger; the density part gives w [F, H_MO] and the model term
      L_mk += w (f_m conj(V_km) - f_k V_mk).
    printed_indices=True uses f_k conj(V_km) - f_m V_mk instead (the index placement
    as printed), which the finite-difference pins reject."""
    assert wl.kind == "complex_full"
    Cs, ds = _densities(wl, params)
    ns = _hubbard_density(wl, ds)
    E = energy_odd(wl, params, lam)
    grads = []
    for inst, a, C, n in zip(wl.instances, params, Cs, ns):
        H = _hamiltonian(inst, n, wl.hubbard_U)
        H_MO = C.conj().T @ H @ C
        F = np.diag(inst.f)
        # with an overlap C = C0 exp(A) on orthonormalized sites is S^(1/2) C0 exp(A), and
        # S^(1/2) C0 is orthonormal: the term's part of L keeps its form with S^(1/2) C
        V = orbital_potential_elements(_lowdin_orbitals(inst, C), lam)
        f = inst.f
        if printed_indices:
            odd = f[None, :] * V.T.conj() - f[:, None] * V
        else:
            odd = f[:, None] * V.T.conj() - f[None, :] * V
        L = inst.weight * (F @ H_MO - H_MO @ F + odd)
        w, Vec = eig_iA(generator(wl.kind, a))
        Lt = Vec.conj().T @ L @ Vec
        Y = Vec @ (Lt * divided_difference_factor(w)) @ Vec.conj().T
        M = L.shape[0]
        delta = np.eye(M)
        dEda = 0.5 * (2.0 - delta) * Y.T
        dRe = 2.0 * np.real(dEda)
        dIm = -2.0 * np.imag(dEda)
        grads.append(np.triu(dRe, 1) + 1j * np.triu(dIm))
    return E, grads


def density_matrices(wl, params) -> List[np.ndarray]:
    """rho = C F C^dagger per instance, C = C0 exp(A) (Sec. 2, the density matrix of the
    orbitals and their occupations; k-point weights not applied)."""
    out = []
    for inst, a in zip(wl.instances, params):
        C = inst.C0 @ expm_eig(generator(wl.kind, a))
        out.append((C * inst.f[None, :]) @ C.conj().T)
    return out


def unitary(wl, params) -> List[np.ndarray]:
    """exp(A) per instance (the etdm_expm output)."""
    return [expm_eig(generator(wl.kind, a)) for a in params]


def bch_series_Y(A: np.ndarray, L: np.ndarray, terms: int = 60) -> np.ndarray:
    """Eq. grad_expansion: L + [A, L]/2! + [A, [A, L]]/3! + ... (a cross-check of Y)."""
    out = L.copy()
    term = L.copy()
    fact = 1.0
    for k in range(1, terms):
        term = A @ term - term @ A
        fact *= (k + 1)
        out = out + term / fact
    return out


def y_matrix(wl, params, idx: int) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """(A, L, Y) for one instance, for pins on Y itself."""
    Cs, ds = _densities(wl, params)
    ns = _hubbard_density(wl, ds)
    inst, a, C, n = wl.instances[idx], params[idx], Cs[idx], ns[idx]
    A = generator(wl.kind, a)
    H = _hamiltonian(inst, n, wl.hubbard_U)
    H_MO = C.conj().T @ H @ C
    F = np.diag(inst.f)
    L = inst.weight * (F @ H_MO - H_MO @ F)
    w, V = eig_iA(A)
    Y = V @ ((V.conj().T @ L @ V) * divided_difference_factor(w)) @ V.conj().T
    return A, L, Y


# ----------------------------------------------------------------------------
# structured occupied-virtual path (real B, binary occupations)
# ----------------------------------------------------------------------------

_GL_NODES = 48


def _gauss_legendre_01(sig_max: float = 0.0):
    """Composite Gauss-Legendre rule on [0, 1] for the pair integrals.  Their integrands
    are products of two oscillations, so their frequency is at most 2 sig_max: the
    interval is cut into pieces over which that phase advances by at most 40 rad, with
    48 nodes per piece (a 48-node rule is exact to rounding for phases well beyond 40)."""
    pieces = max(1, int(np.ceil(2.0 * max(float(sig_max), 0.0) / 40.0)))
    x, wq = np.polynomial.legendre.leggauss(_GL_NODES)
    h = 1.0 / pieces
    t = ((np.arange(pieces)[:, None] + 0.5 * (x[None, :] + 1.0)) * h).ravel()
    return t, np.tile(0.5 * h * wq, pieces)


def ov_pair_integrals(sig: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """The two pair integrals of the structured gradient, by Gauss-Legendre quadrature:

      mu1[k, l] = -integral_0^1 (t^2/2) cos(t s_k) sinc(t s_l / 2)^2 dt
      mu2[k, l] =  integral_0^1 t^2 sinc(t s_k) sinc(t s_l) dt

    with s = singular values of B.  Both integrands are entire; the composite rule grows
    with the largest angle, so any rotation angle is covered.
    """
    t, wq = _gauss_legendre_01(sig.max() if sig.size else 0.0)
    ts = t[None, :] * sig[:, None]  # [N, nodes]
    cos_t = np.cos(ts)
    sinc_t = _sinc(ts)
    sinc_half2 = _sinc(0.5 * ts) ** 2
    mu1 = -(cos_t * (wq * t ** 2 / 2.0)[None, :]) @ sinc_half2.T
    mu2 = (sinc_t * (wq * t ** 2)[None, :]) @ sinc_t.T
    return mu1, mu2


def energy_grad_ov(inst, B: np.ndarray, hubbard_U: float, want_parts: bool = False, progress=None):
    """E and dE/dB for one real instance with A = [[0, B], [-B^T, 0]] and binary f.

    Derived from Eq. gradients with the singular-value basis of B: in the basis
    blockdiag(X, [Z, Z_perp]) with B = X diag(s) Z^T, A is a set of independent
    2 x 2 plane rotations by s_k; integrating exp(tA) L exp(-tA) over t blockwise
    and returning to the original basis gives

      Y_ov = sinc(sqrt P) L_ov + X Nm X^T B,   Gam = X^T L_ov B^T X,
      Nm[k, l] = Gam[k, l] mu1[k, l] + Gam[l, k] mu2[k, l],
      dE/dB = -2 Y_ov.

    H0 may be dense or block-sparse (scipy.sparse is used for the product).  progress,
    if given, is called with a short message after each large step (long runs report
    where they are).
    """
    note = progress or (lambda msg: None)
    N, Nv = B.shape
    M = N + Nv
    assert inst.S is None, "the structured path takes an orthonormal basis"
    f_occ = float(inst.f[0])
    assert np.all(inst.f[:N] == f_occ) and np.all(inst.f[N:] == 0.0)
    s, X = np.linalg.eigh(B @ B.T)
    sig = np.sqrt(np.clip(s, 0.0, None))
    note("oracle: eigendecomposition of B B^T")
    cosP = (X * np.cos(sig)) @ X.T
    sincP = (X * _sinc(sig)) @ X.T
    WP = (X * (-0.5 * _sinc(0.5 * sig) ** 2)) @ X.T
    C0o, C0v = inst.C0[:, :N], inst.C0[:, N:]
    Q1 = C0v @ B.T
    note("oracle: C0_v B^T")
    Cocc = C0o @ cosP - Q1 @ sincP
    Cvirt = C0v + (C0o @ sincP + Q1 @ WP) @ B
    note("oracle: rotated orbitals")
    d = f_occ * (Cocc ** 2).sum(axis=1)
    T0 = _h0_times(inst, Cocc)
    E = f_occ * float((Cocc * T0).sum()) + 0.5 * hubbard_U * float((d ** 2).sum())
    T = T0 + hubbard_U * d[:, None] * Cocc
    Lov = f_occ * (T.T @ Cvirt)
    note("oracle: L_ov")
    Gam = X.T @ (Lov @ B.T) @ X
    mu1, mu2 = ov_pair_integrals(sig)
    Nm = Gam * mu1 + Gam.T * mu2
    g = -2.0 * (sincP @ Lov + X @ Nm @ (X.T @ B))
    if want_parts:
        return E, g, dict(Cocc=Cocc, Cvirt=Cvirt, d=d, Lov=Lov, sig=sig, X=X)
    return E, g


def energy_grad_ov_approx(inst, B: np.ndarray, hubbard_U: float):
    """E and the approximate gradient of Eq. app_grad for one real occupied-virtual
    instance: with G ~ L^T, the ov parameters get g = -2 L_ov, L_ov = f_occ C_occ^T H C_virt
    (the structured form of energy_grad_approx, for sizes where the M x M definition
    path is out of reach)."""
    E, _, parts = energy_grad_ov(inst, B, hubbard_U, want_parts=True)
    return E, -2.0 * parts["Lov"]


def _h0_times(inst, Cm: np.ndarray) -> np.ndarray:
    if inst.H0 is not None:
        return inst.H0 @ Cm
    import scipy.sparse as sp
    b = inst.H0_bsr
    Hs = sp.bsr_matrix((b.blocks, b.col_idx, b.row_ptr), shape=(b.n, b.n))
    return Hs @ Cm


def energy_grad_ov_workload(wl, params) -> Tuple[float, List[np.ndarray]]:
    assert wl.kind == "real_ov" and not wl.couple
    E = 0.0
    gs = []
    for inst, B in zip(wl.instances, params):
        e, g = energy_grad_ov(inst, B, wl.hubbard_U)
        E += e
        gs.append(g)
    return E, gs


# ----------------------------------------------------------------------------
# helpers for the optimizer and tests
# ----------------------------------------------------------------------------


def zero_params(wl) -> List[np.ndarray]:
    if wl.kind == "real_ov":
        return [np.zeros((inst.N, inst.M - inst.N)) for inst in wl.instances]
    return [np.zeros((inst.M, inst.M), dtype=np.complex128) for inst in wl.instances]


def parity_params(wl) -> List[np.ndarray]:
    if wl.kind == "real_ov":
        return [inst.A.copy() for inst in wl.instances]
    return [np.triu(inst.A) for inst in wl.instances]


def orbital_energies(wl) -> List[np.ndarray]:
    """eps_i = diag(C0^dagger H(rho0) C0), computed once at the start (Sec. 3.3)."""
    ps = zero_params(wl)
    Cs, ds = _densities(wl, ps)
    ns = _hubbard_density(wl, ds)
    out = []
    for inst, C, n in zip(wl.instances, Cs, ns):
        H = _hamiltonian(inst, n, wl.hubbard_U)
        out.append(np.real(np.diag(C.conj().T @ H @ C)))
    return out


def flatten(kind: str, xs: Sequence[np.ndarray]) -> np.ndarray:
    """Real vector of the free variables (Sec. 3: Re of the strict upper triangle,
    then Im of the upper triangle incl. the diagonal, per k-point)."""
    parts = []
    for x in xs:
        if kind == "real_ov":
            parts.append(x.ravel())
        else:
            M = x.shape[0]
            iu = np.triu_indices(M, 1)
            iu0 = np.triu_indices(M, 0)
            parts.append(np.real(x[iu]))
            parts.append(np.imag(x[iu0]))
    return np.concatenate(parts) if parts else np.zeros(0)


def unflatten(kind: str, wl, v: np.ndarray) -> List[np.ndarray]:
    out = []
    o = 0
    for inst in wl.instances:
        M, N = inst.M, inst.N
        if kind == "real_ov":
            n = N * (M - N)
            out.append(v[o:o + n].reshape(N, M - N).copy())
            o += n
        else:
            iu = np.triu_indices(M, 1)
            iu0 = np.triu_indices(M, 0)
            x = np.zeros((M, M), dtype=np.complex128)
            x[iu] = v[o:o + iu[0].size]
            o += iu[0].size
            x[iu0] += 1j * v[o:o + iu0[0].size]
            o += iu0[0].size
            out.append(x)
    return out
