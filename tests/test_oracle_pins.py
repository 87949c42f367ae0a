"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: an
independent algorithm, a hand-derived closed form, an invariance, finite
differences, a series expansion, or a brute-force minimum.
"""
import copy

import numpy as np
import pytest
import scipy.optimize

from oracle import etdm as O
from oracle import lbfgs as LB
from oracle import scf
from workloads import Instance, Workload, make_config, tiny_complex, tiny_real
from workloads.gen import chain_hamiltonian, haar_orthogonal, rng_for


def rand_skew_hermitian(M, rng, scale=0.7, real=False):
    X = rng.standard_normal((M, M)) * scale
    if not real:
        X = X + 1j * rng.standard_normal((M, M)) * scale
    return 0.5 * (X - X.conj().T)


# ---------------------------------------------------------------------------
# matrix exponential (Eq. ed, Eq. uinv)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("M,real", [(1, False), (2, True), (7, False), (16, True), (33, False)])
def test_expm_unitary_det_and_pade(M, real):
    rng = np.random.default_rng(M)
    A = rand_skew_hermitian(M, rng, real=real)
    U = O.expm_eig(A)
    assert np.abs(U.conj().T @ U - np.eye(M)).max() < 1e-14 * M
    # det exp(A) = exp(Tr A): +1 for real A, unit modulus in general
    assert abs(np.linalg.det(U) - np.exp(np.trace(A))) < 1e-13 * M
    # independent algorithm: scaling and squaring with Pade (Eq. ss)
    assert np.abs(U - O.expm_pade(A)).max() < 1e-13 * M


def test_expm_plane_rotation_closed_form():
    for th in (0.0, 1e-9, 0.3, -1.2, 3.0, 7.5):
        A = np.array([[0.0, th], [-th, 0.0]])
        U = O.expm_eig(A)
        ref = np.array([[np.cos(th), np.sin(th)], [-np.sin(th), np.cos(th)]])
        assert np.abs(U - ref).max() < 1e-15 * max(1.0, abs(th))


@pytest.mark.parametrize("N,Nv,scale", [(3, 5, 0.4), (5, 3, 0.4), (4, 4, 1.5), (1, 6, 0.0),
                                         (6, 2, 2.0), (16, 48, 0.05)])
def test_hutter_closed_form_matches_eigh(N, Nv, scale):
    """Corrected Eq. uinv equals Eq. ed, including N > Nv (rank-deficient P) and B = 0."""
    B = np.random.default_rng(N * 10 + Nv).standard_normal((N, Nv)) * scale
    U1 = O.expm_ov(B)
    U2 = O.expm_eig(O.ov_generator(B))
    assert np.abs(U1 - U2).max() < 1e-14 * (N + Nv)
    assert np.abs(U1.T @ U1 - np.eye(N + Nv)).max() < 1e-14 * (N + Nv)


def test_hutter_as_printed_is_not_exp():
    """Reading of the garbled Eq. uinv: cos(P) in the top-left block (as printed)
    is not the exponential; cos(P^{1/2}) is."""
    B = np.random.default_rng(3).standard_normal((3, 4)) * 0.8
    U = O.expm_eig(O.ov_generator(B))
    s, X = np.linalg.eigh(B @ B.T)
    printed_top_left = (X * np.cos(s)) @ X.T
    assert np.abs(printed_top_left - U[:3, :3]).max() > 1e-2


# ---------------------------------------------------------------------------
# energy and gradient
# ---------------------------------------------------------------------------

def two_level_workload(a, b, c, U_hub):
    H0 = np.array([[a, b], [b, c]])
    inst = Instance(M=2, N=1, f=np.array([2.0, 0.0]), C0=np.eye(2), A=np.zeros((1, 1)), H0=H0)
    return Workload(0, "two-level", "real_ov", U_hub, False, [inst])


@pytest.mark.parametrize("th", [0.0, 0.2, -0.7, 1.3, 2.9])
def test_two_level_closed_form(th):
    """Hand-derived: orbital (cos th, -sin th), E = 2 <H0> + U/2 (n1^2 + n2^2),
    dE/dth = 2 (c - a) sin 2th - 4 b cos 2th - 2 U sin 4th."""
    a, b, c, Uh = -0.7, 0.3, 0.9, 0.5
    wl = two_level_workload(a, b, c, Uh)
    E, g = O.energy_grad(wl, [np.array([[th]])])
    cs, sn = np.cos(th), np.sin(th)
    E_ref = 2 * (a * cs * cs - 2 * b * cs * sn + c * sn * sn) + 0.5 * Uh * ((2 * cs * cs) ** 2 + (2 * sn * sn) ** 2)
    g_ref = 2 * (c - a) * np.sin(2 * th) - 4 * b * np.cos(2 * th) - 2 * Uh * np.sin(4 * th)
    assert abs(E - E_ref) < 1e-14
    assert abs(g[0][0, 0] - g_ref) < 1e-14
    E2, g2 = O.energy_grad_ov_workload(wl, [np.array([[th]])])
    assert abs(E2 - E_ref) < 1e-14 and abs(g2[0][0, 0] - g_ref) < 1e-14


def test_energy_at_zero_equals_reference_density():
    wl = tiny_real(10, 3, seed=4)
    inst = wl.instances[0]
    rho0 = inst.C0 @ np.diag(inst.f) @ inst.C0.T
    n = np.diag(rho0)
    E_ref = np.sum(rho0 * inst.H0) + 0.5 * wl.hubbard_U * np.sum(n ** 2)
    assert abs(O.energy(wl, O.zero_params(wl)) - E_ref) < 1e-13 * abs(E_ref)


def _as_complex_full(wl):
    w = copy.deepcopy(wl)
    w.kind = "complex_full"
    for inst in w.instances:
        inst.C0 = inst.C0.astype(np.complex128)
        inst.H0 = inst.H0.astype(np.complex128)
    return w


def test_occupied_occupied_invariance():
    """For a unitary-invariant functional with equal occupations, rotations inside
    the occupied (or virtual) block leave E unchanged (Sec. 3.4)."""
    wl = _as_complex_full(tiny_real(9, 4, seed=2))
    rng = np.random.default_rng(0)
    A = np.zeros((9, 9), dtype=np.complex128)
    A[:4, :4] = rand_skew_hermitian(4, rng, 0.8)
    A[4:, 4:] = rand_skew_hermitian(5, rng, 0.8)
    E0 = O.energy(wl, O.zero_params(wl))
    assert abs(O.energy(wl, [np.triu(A)]) - E0) < 1e-13 * abs(E0)


def test_gauge_covariance_of_ov_gradient():
    """E(C0 W, Voo^T B Vvv) = E(C0, B) and g' = Voo^T g Vvv for W = blockdiag(Voo, Vvv)."""
    wl = tiny_real(11, 4, seed=5, scale=0.3)
    B = wl.instances[0].A
    E, (g,) = O.energy_grad(wl, [B])
    rng = np.random.default_rng(1)
    Voo = haar_orthogonal(4, rng)
    Vvv = haar_orthogonal(7, rng)
    W = np.zeros((11, 11))
    W[:4, :4], W[4:, 4:] = Voo, Vvv
    wl2 = copy.deepcopy(wl)
    wl2.instances[0].C0 = wl.instances[0].C0 @ W
    E2, (g2,) = O.energy_grad(wl2, [Voo.T @ B @ Vvv])
    assert abs(E2 - E) < 1e-13 * abs(E)
    assert np.abs(g2 - Voo.T @ g @ Vvv).max() < 1e-13 * np.abs(g).max()


def test_gradient_at_zero_is_commutator():
    """At A = 0 the gradient is L^T exactly (Eq. app_grad): dE/dB_ij = -2 f_occ (H_MO)_{i,N+j}."""
    wl = tiny_real(12, 5, seed=7)
    inst = wl.instances[0]
    E, (g,) = O.energy_grad(wl, O.zero_params(wl))
    rho0 = inst.C0 @ np.diag(inst.f) @ inst.C0.T
    H = inst.H0 + wl.hubbard_U * np.diag(np.diag(rho0))
    H_MO = inst.C0.T @ H @ inst.C0
    assert np.abs(g - (-2.0 * 2.0 * H_MO[:5, 5:])).max() < 1e-14


# ---------------------------------------------------------------------------
# approximate gradient G ~ L^T (Eq. app_grad)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("kind", ["real_ov", "complex"])
def test_approx_gradient_at_zero_matches_finite_differences(kind):
    """At A = 0 the first term of the expansion is the whole gradient: G ~ L^T agrees
    with central differences of E (not only with the exact-gradient code)."""
    wl = tiny_real(11, 4, seed=21) if kind == "real_ov" else tiny_complex(6, nk_side=1, kT=0.05)
    zero = O.zero_params(wl)
    _, grads = O.energy_grad_approx(wl, zero)
    gv = O.flatten(wl.kind, grads)
    _, gex = O.energy_grad(wl, zero)
    assert np.abs(gv - O.flatten(wl.kind, gex)).max() < 1e-13 * (np.abs(gv).max() + 1.0)
    rng = np.random.default_rng(22)
    for _ in range(3):
        d = rng.standard_normal(gv.size)
        assert abs(_fd_directional(wl, zero, d, 1e-3) - gv @ d) < 2e-9 * (np.abs(gv).sum() + 1.0)


@pytest.mark.parametrize("kind,order", [("real_ov", 2), ("complex", 1)])
def test_approx_gradient_error_order(kind, order):
    """G ~ L^T drops the terms of the expansion beyond the first; the next one is
    [A, L]/2.  With fractional occupations (complex case) it is O(A), so the error
    halves with A.  In the ov parametrization with integer occupations A and L are
    both block off-diagonal, [A, L] has no ov block, and the error is O(A^2)."""
    wl = tiny_real(12, 5, seed=23, scale=1.0) if kind == "real_ov" else tiny_complex(6, nk_side=1, kT=0.05)
    base = O.parity_params(wl)
    errs = []
    for t in (0.04, 0.02, 0.01):
        p = [t * b / max(np.abs(b).max(), 1e-300) for b in base]
        _, ga = O.energy_grad_approx(wl, p)
        _, ge = O.energy_grad(wl, p)
        errs.append(np.linalg.norm(O.flatten(wl.kind, ga) - O.flatten(wl.kind, ge)))
    want = 2.0 ** order
    assert all(0.9 * want < errs[i] / errs[i + 1] < 1.1 * want for i in range(2)), errs
    assert errs[2] > 0.0


def test_approx_gradient_exact_for_one_rotation_plane():
    """One occupied and one virtual orbital: rotations in the single plane commute,
    so the derivative at the current orbitals, L^T, is the exact dE/dtheta for
    every angle (closed form E(theta) differentiated numerically)."""
    M, N = 2, 1
    rng = np.random.default_rng(24)
    H0 = rng.standard_normal((M, M))
    H0 = 0.5 * (H0 + H0.T)
    C0 = haar_orthogonal(M, rng)
    wl = Workload(0, "two-level", "real_ov", 0.7, False)
    f = np.array([2.0, 0.0])
    for th in (0.3, -1.1, 2.0):
        wl.instances = [Instance(M=M, N=N, f=f, C0=C0, A=np.array([[th]]), H0=H0)]
        _, (ga,) = O.energy_grad_approx(wl, [np.array([[th]])])
        _, (ge,) = O.energy_grad(wl, [np.array([[th]])])
        h = 1e-4
        fd = (O.energy(wl, [np.array([[th + h]])]) - O.energy(wl, [np.array([[th - h]])])) / (2 * h)
        assert abs(ga[0, 0] - ge[0, 0]) < 1e-12 * max(1.0, abs(ge[0, 0]))
        assert abs(ga[0, 0] - fd) < 1e-7 * max(1.0, abs(fd))


def test_structured_approx_gradient_matches_definition_path():
    """The structured ov form (g = -2 L_ov from C_occ, C_virt) agrees with the M x M
    definition path of G ~ L^T at a rotation far from zero."""
    wl = tiny_real(14, 5, seed=25, scale=0.8)
    p = O.parity_params(wl)
    E, (g,) = O.energy_grad_approx(wl, p)
    Es, gs = O.energy_grad_ov_approx(wl.instances[0], p[0], wl.hubbard_U)
    assert abs(E - Es) < 1e-12 * max(1.0, abs(E))
    assert np.abs(g - gs).max() < 1e-12 * max(1.0, np.abs(g).max())
    _, (ge,) = O.energy_grad(wl, p)
    assert np.abs(g - ge).max() > 1e-6  # far enough from zero that the two gradients differ


def _pade_from_conditions(m):
    """[m/m] Pade approximant of exp from its definition, in exact rationals:
    q(x) e^x - p(x) = O(x^(2m+1)) with q_0 = 1 (m linear equations for q_1..q_m from the
    coefficients of x^(m+1)..x^(2m), then p_k = sum_j q_j / (k - j)!)."""
    from fractions import Fraction
    from math import factorial

    def inv_fact(n):
        return Fraction(1, factorial(n)) if n >= 0 else Fraction(0)
    # rows k = m+1..2m: sum_{j=1..m} q_j / (k-j)! = -1 / k!
    rows = [[inv_fact(k - j) for j in range(1, m + 1)] + [-inv_fact(k)] for k in range(m + 1, 2 * m + 1)]
    for c in range(m):  # Gauss-Jordan in exact arithmetic
        piv = next(r for r in range(c, m) if rows[r][c] != 0)
        rows[c], rows[piv] = rows[piv], rows[c]
        rows[c] = [v / rows[c][c] for v in rows[c]]
        for r in range(m):
            if r != c and rows[r][c] != 0:
                f = rows[r][c]
                rows[r] = [v - f * w for v, w in zip(rows[r], rows[c])]
    q = [Fraction(1)] + [rows[j][m] for j in range(m)]
    p = [sum(q[j] * inv_fact(k - j) for j in range(0, k + 1)) for k in range(m + 1)]
    return p, q


def test_pade_coefficients_match_the_defining_conditions():
    """The closed-form b_j of every tabulated degree equal the approximant solved from its
    defining conditions, and the denominator is p(-x); [3/3] is 1 + x/2 + x^2/10 + x^3/120."""
    assert np.allclose(O.pade_coefficients(3), [1.0, 0.5, 0.1, 1.0 / 120.0], rtol=0, atol=1e-16)
    for m, _ in O.PADE_THETA:
        p, q = _pade_from_conditions(m)
        b = O.pade_coefficients(m)
        for j in range(m + 1):
            assert abs(b[j] - float(p[j])) <= 1e-15 * float(p[j]), (m, j)
            assert q[j] == (-1) ** j * p[j], (m, j)


@pytest.mark.parametrize("theta,m,s", [(0.01, 3, 0), (0.2, 5, 0), (0.9, 7, 0), (2.0, 9, 0), (5.0, 13, 0),
                                       (40.0, 13, 3), (1000.0, 13, 8)])
def test_expm_ss_plane_rotation(theta, m, s):
    """exp([[0, t], [-t, 0]]) is the rotation by t; the 1-norm t picks degree m and s halvings."""
    A = np.array([[0.0, theta], [-theta, 0.0]])
    assert O.pade_degree_and_scaling(theta) == (m, s)
    R = O.expm_ss(A)
    ref = np.array([[np.cos(theta), np.sin(theta)], [-np.sin(theta), np.cos(theta)]])
    assert np.abs(R - ref).max() < 1e-13 * max(1.0, 2.0 ** s)


def test_expm_ss_closed_forms():
    """Nilpotent N (N^5 = 0): exp(N) = sum_k<5 N^k / k!; diagonal i w: exp is diag(e^{i w})."""
    rng = np.random.default_rng(31)
    N = np.triu(rng.standard_normal((5, 5)), 1) * 3.0
    ref = np.eye(5)
    term = np.eye(5)
    for k in range(1, 5):
        term = term @ N / k
        ref = ref + term
    assert np.abs(O.expm_ss(N) - ref).max() < 1e-12 * np.abs(ref).max()
    w = rng.uniform(-9.0, 9.0, 7)
    D = O.expm_ss(np.diag(1j * w))
    assert np.abs(D - np.diag(np.exp(1j * w))).max() < 1e-13


@pytest.mark.parametrize("scale", [1e-3, 0.3, 3.0, 60.0])
def test_expm_ss_matches_eigendecomposition_and_scipy(scale):
    """Random skew-Hermitian A: expm_ss agrees with exp through eigh(iA) and with SciPy's
    expm, and is unitary."""
    rng = np.random.default_rng(32)
    M = 40
    X = rng.standard_normal((M, M)) + 1j * rng.standard_normal((M, M))
    A = scale * (X - X.conj().T) / np.sqrt(M)
    R = O.expm_ss(A)
    tol = 1e-13 * max(1.0, scale)
    assert np.abs(R - O.expm_eig(A)).max() < tol
    assert np.abs(R - O.expm_pade(A)).max() < tol
    assert np.abs(R.conj().T @ R - np.eye(M)).max() < tol


def test_scaling_and_squaring_configuration_matches_eigendecomposition():
    """E and G ~ L^T with exp(A) by scaling and squaring equal those with exp(A) through
    eigh(iA), also for rotations large enough to need squarings."""
    wl = tiny_complex(9, nk_side=2, kT=0.2)
    for scale in (1.0, 40.0):
        p = [scale * a for a in O.parity_params(wl)]
        E1, G1 = O.energy_grad_approx(wl, p)
        E2, G2 = O.energy_grad_approx(wl, p, expm=O.expm_ss)
        assert abs(E1 - E2) < 1e-12 * max(1.0, abs(E1))
        assert max(np.abs(a - b).max() for a, b in zip(G1, G2)) < 1e-11 * max(1.0, scale)


@pytest.mark.parametrize("scale", [0.01, 1.0, 20.0])
def test_frechet_expm_ss(scale):
    """The Frechet derivative from scaling and squaring equals the upper-right block of
    exp([[A, E], [0, A]]) (through eigh-free SciPy expm of the doubled matrix), SciPy's
    expm_frechet, and a central difference of expm_ss."""
    rng = np.random.default_rng(33)
    M = 12
    X = rng.standard_normal((M, M)) + 1j * rng.standard_normal((M, M))
    A = scale * (X - X.conj().T) / np.sqrt(M)
    E = rng.standard_normal((M, M)) + 1j * rng.standard_normal((M, M))
    U, L = O.frechet_expm_ss(A, E)
    big = np.block([[A, E], [np.zeros_like(A), A]])
    ref = scipy.linalg.expm(big)[:M, M:]
    tol = 1e-12 * max(1.0, scale)
    assert np.abs(U - O.expm_ss(A)).max() < 1e-14 * max(1.0, scale)
    assert np.abs(L - ref).max() < tol * np.abs(ref).max()
    assert np.abs(L - scipy.linalg.expm_frechet(A, E, compute_expm=False)).max() < tol * np.abs(ref).max()
    h = 1e-5
    fd = (O.expm_ss(A + h * E) - O.expm_ss(A - h * E)) / (2 * h)
    assert np.abs(L - fd).max() < 1e-7 * np.abs(ref).max()


def test_exact_gradient_by_scaling_and_squaring():
    """Y = L(A, L) exp(A)^dagger reproduces the eigenbasis gradient (complex, fractional
    occupations, coupled k-points) also for rotations that need squarings."""
    wl = tiny_complex(9, nk_side=2, kT=0.2)
    for scale in (1.0, 30.0):
        p = [scale * a for a in O.parity_params(wl)]
        E1, G1 = O.energy_grad(wl, p)
        E2, G2 = O.energy_grad_ss(wl, p)
        assert abs(E1 - E2) < 1e-12 * max(1.0, abs(E1))
        assert max(np.abs(a - b).max() for a, b in zip(G1, G2)) < 1e-11 * max(1.0, scale)


def _fd_odd(wl, params, lam, d, h=1e-3):
    """Richardson central difference of energy_odd along d (flat free variables)."""
    v = O.flatten(wl.kind, params)

    def E(t):
        return O.energy_odd(wl, O.unflatten(wl.kind, wl, v + t * d), lam)
    d1 = (E(h) - E(-h)) / (2 * h)
    d2 = (E(h / 2) - E(-h / 2)) / h
    return (4 * d2 - d1) / 3


def test_orbital_dependent_gradient_matches_finite_differences():
    """The L of the orbital-dependent model term, derived as G - G^dagger, gives the
    finite-difference gradient (fractional occupations, coupled k-points, far from
    A = 0); the index placement as printed does not; lam = 0 is energy_grad."""
    wl = tiny_complex(7, nk_side=2, kT=0.3)
    p = [3.0 * a for a in O.parity_params(wl)]
    lam = 0.7
    E, G = O.energy_grad_odd(wl, p, lam)
    _, Gp = O.energy_grad_odd(wl, p, lam, printed_indices=True)
    g, gp = O.flatten(wl.kind, G), O.flatten(wl.kind, Gp)
    rng = np.random.default_rng(41)
    worst_printed = 0.0
    for _ in range(4):
        d = rng.standard_normal(g.size)
        fd = _fd_odd(wl, p, lam, d)
        assert abs(fd - g @ d) < 1e-8 * (np.abs(g).sum() + 1.0), (fd, g @ d)
        worst_printed = max(worst_printed, abs(fd - gp @ d))
    assert worst_printed > 1e-3
    E0, G0 = O.energy_grad_odd(wl, p, 0.0)
    E1, G1 = O.energy_grad(wl, p)
    assert abs(E0 - E1) < 1e-12 and max(np.abs(a - b).max() for a, b in zip(G0, G1)) < 1e-13
    # not invariant under rotations among the occupied orbitals (the ov form cannot carry it)
    inst = wl.instances[0]
    occ = np.flatnonzero(inst.f > 0.5)
    a = np.zeros((inst.M, inst.M), dtype=complex)
    a[occ[0], occ[1]] = 0.4
    zero = O.zero_params(wl)
    rot = [a] + zero[1:]
    assert abs(O.energy_odd(wl, rot, lam) - O.energy_odd(wl, zero, lam)) > 1e-6


@pytest.mark.parametrize("overlap", [False, True])
def test_approx_gradient_with_orbital_term_is_exact_at_zero(overlap):
    """G ~ L^T with the orbital-dependent term: at A = 0 every divided-difference factor
    is 1, so it equals the exact gradient of energy_grad_odd (pinned by finite
    differences), with and without an overlap; away from A = 0 the two differ."""
    from workloads import with_overlap
    wl = tiny_complex(7, nk_side=2, kT=0.3)
    if overlap:
        wl = with_overlap(wl)
    lam = 0.7
    zero = O.zero_params(wl)
    Ea, Ga = O.energy_grad_approx(wl, zero, lam=lam)
    Ee, Ge = O.energy_grad_odd(wl, zero, lam)
    assert abs(Ea - Ee) < 1e-13 * max(1.0, abs(Ee))
    assert max(np.abs(a - b).max() for a, b in zip(Ga, Ge)) < 1e-13
    assert max(np.abs(g).max() for g in Ge) > 1e-3
    p = [3.0 * a for a in O.parity_params(wl)]
    _, Ga = O.energy_grad_approx(wl, p, lam=lam)
    _, Ge = O.energy_grad_odd(wl, p, lam)
    assert max(np.abs(a - b).max() for a, b in zip(Ga, Ge)) > 1e-3


def test_orbital_dependent_gradient_with_overlap_matches_finite_differences():
    """In a non-orthogonal basis the model term uses the Lowdin coefficients S^(1/2) C;
    its gradient still matches finite differences, and the term differs from one built
    on the raw coefficients."""
    from workloads import with_overlap
    wl = with_overlap(tiny_complex(7, nk_side=2, kT=0.3))
    p = [2.0 * a for a in O.parity_params(wl)]
    lam = 0.7
    E, G = O.energy_grad_odd(wl, p, lam)
    g = O.flatten(wl.kind, G)
    rng = np.random.default_rng(43)
    for _ in range(4):
        d = rng.standard_normal(g.size)
        fd = _fd_odd(wl, p, lam, d)
        assert abs(fd - g @ d) < 1e-8 * (np.abs(g).sum() + 1.0), (fd, g @ d)
    Cs, _ = O._densities(wl, p)
    raw = sum(-0.5 * lam * inst.weight * float((inst.f[None, :] * np.abs(C) ** 4).sum())
              for inst, C in zip(wl.instances, Cs))
    assert abs((E - O.energy(wl, p)) - raw) > 1e-6


@pytest.mark.parametrize("kind", ["real_ov", "complex"])
def test_non_orthogonal_basis_gradient_matches_finite_differences(kind):
    """With an overlap S != I (C0^H S C0 = I) the energy uses Lowdin populations and
    H = H0 + U S^(1/2) diag(n) S^(1/2); the gradient matches finite differences, the
    orbitals stay S-orthonormal, and at A = 0 E is Tr(rho H0) + U/2 |n|^2 from the
    inputs directly."""
    from workloads import with_overlap
    wl = with_overlap(tiny_real(11, 4, seed=21, scale=0.4) if kind == "real_ov"
                      else tiny_complex(6, nk_side=1, kT=0.2))
    p = O.parity_params(wl)
    E, G = O.energy_grad(wl, p)
    g = O.flatten(wl.kind, G)
    rng = np.random.default_rng(42)
    for _ in range(3):
        d = rng.standard_normal(g.size)
        assert abs(_fd_directional(wl, p, d, 1e-3) - g @ d) < 1e-8 * (np.abs(g).sum() + 1.0)
    inst = wl.instances[0]
    C = inst.C0 @ O.expm_eig(O.generator(wl.kind, p[0]))
    assert np.abs(C.conj().T @ inst.S @ C - np.eye(inst.M)).max() < 1e-13
    # A = 0 by hand: rho0 = C0 F C0^H, n = diag(S^1/2 rho0 S^1/2) with S^1/2 from scipy
    S_half = scipy.linalg.sqrtm(inst.S)
    rho0 = inst.C0 @ np.diag(inst.f) @ inst.C0.conj().T
    n = np.real(np.diag(S_half @ rho0 @ S_half))
    E0 = float(np.real(np.trace(rho0 @ inst.H0))) * inst.weight + 0.5 * wl.hubbard_U * float(n @ n)
    if len(wl.instances) == 1:
        assert abs(O.energy(wl, O.zero_params(wl)) - E0) < 1e-12 * max(1.0, abs(E0))


def _fd_directional(wl, params, d, h):
    kind = wl.kind
    v = O.flatten(kind, params)

    def E(t):
        return O.energy(wl, O.unflatten(kind, wl, v + t * d))
    # Richardson-extrapolated central difference (error O(h^4))
    d1 = (E(h) - E(-h)) / (2 * h)
    d2 = (E(h / 2) - E(-h / 2)) / h
    return (4 * d2 - d1) / 3


@pytest.mark.parametrize("case", ["real_ov", "real_ov_rankdef", "complex_fd_coupled", "complex_integer"])
def test_gradient_matches_finite_differences(case):
    if case == "real_ov":
        wl = tiny_real(13, 4, seed=8, scale=0.35)
    elif case == "real_ov_rankdef":
        wl = tiny_real(7, 5, seed=9, scale=0.5)
    elif case == "complex_fd_coupled":
        wl = tiny_complex(8, nk_side=2, kT=0.3)
        for inst in wl.instances:
            inst.A = inst.A * 6.0  # larger rotations than the parity point
    else:
        wl = tiny_complex(6, nk_side=1, kT=0.01)
    params = O.parity_params(wl)
    E, grads = O.energy_grad(wl, params)
    gv = O.flatten(wl.kind, grads)
    rng = np.random.default_rng(11)
    for _ in range(3):
        d = rng.standard_normal(gv.size)
        fd = _fd_directional(wl, params, d, 1e-3)
        assert abs(fd - gv @ d) < 2e-9 * (np.abs(gv).sum() + 1.0)


def test_gradient_per_entry_finite_differences_tiny():
    wl = tiny_real(5, 2, seed=12, scale=0.6)
    params = O.parity_params(wl)
    _, (g,) = O.energy_grad(wl, params)
    for i in range(2):
        for j in range(3):
            d = np.zeros_like(g)
            d[i, j] = 1.0
            fd = _fd_directional(wl, params, d.ravel(), 1e-3)
            assert abs(fd - g[i, j]) < 1e-9


def test_printed_divided_difference_sign_gives_minus_gradient():
    """Reading of Sec. 3.4: D = (exp(-ix) - 1)/(ix) as printed yields -dE/dA; the
    oracle uses D = (1 - exp(-ix))/(ix) = integral_0^1 exp(-itx) dt (Eq. gradients)."""
    wl = tiny_real(8, 3, seed=13, scale=0.4)
    A, L, Y = O.y_matrix(wl, O.parity_params(wl), 0)
    w, V = O.eig_iA(A)
    x = w[:, None] - w[None, :]
    with np.errstate(invalid="ignore", divide="ignore"):
        Dp = np.where(np.abs(x) > 0, (np.exp(-1j * x) - 1.0) / (1j * np.where(x == 0, 1, x)), -1.0)
    Yp = V @ ((V.conj().T @ L @ V) * Dp) @ V.conj().T
    assert np.abs(Yp + Y).max() < 1e-12 * np.abs(Y).max()


@pytest.mark.parametrize("complex_case", [False, True])
def test_y_matches_bch_series(complex_case):
    """Y equals the commutator series of Eq. grad_expansion."""
    wl = tiny_complex(6, nk_side=1, kT=0.2) if complex_case else tiny_real(9, 3, seed=14, scale=0.3)
    A, L, Y = O.y_matrix(wl, O.parity_params(wl), 0)
    if complex_case:
        A, L, Y = O.y_matrix(wl, [p * 8.0 for p in O.parity_params(wl)], 0)
    Ys = O.bch_series_Y(A, L)
    assert np.abs(Ys - Y).max() < 1e-13 * np.abs(Y).max()


@pytest.mark.parametrize("M,N,scale", [(6, 2, 0.5), (7, 5, 0.8), (12, 4, 0.05), (20, 4, 1.0),
                                       (9, 3, 0.0), (30, 6, 2.5)])
def test_structured_ov_equals_dense(M, N, scale):
    wl = tiny_real(M, N, seed=M + N, scale=max(scale, 1e-300))
    if scale == 0.0:
        wl.instances[0].A[:] = 0.0
    p = O.parity_params(wl)
    E, (g,) = O.energy_grad(wl, p)
    E2, (g2,) = O.energy_grad_ov_workload(wl, p)
    assert abs(E - E2) < 1e-13 * abs(E)
    assert np.abs(g - g2).max() < 1e-12 * max(np.abs(g).max(), 1e-300)


def test_pair_integrals_limits_and_closed_forms():
    """mu1, mu2 vs their limits at 0 (-1/6, 1/3) and closed forms away from 0."""
    sig = np.array([0.0, 1e-8, 0.7, 2.3, 7.6])
    mu1, mu2 = O.ov_pair_integrals(sig)
    assert abs(mu1[0, 0] + 1.0 / 6.0) < 1e-15 and abs(mu2[0, 0] - 1.0 / 3.0) < 1e-15
    sk, sl = sig[2:, None], sig[None, 2:]
    sincf = lambda x: np.sinc(x / np.pi)
    Kc = 0.5 * (sincf(sk - sl) + sincf(sk + sl))
    Ks = 0.5 * (sincf(sk - sl) - sincf(sk + sl))
    assert np.abs(mu1[2:, 2:] - (Kc - sincf(sk)) / sl ** 2).max() < 1e-14
    assert np.abs(mu2[2:, 2:] - Ks / (sk * sl)).max() < 1e-14


def _mp_pair_integrals(a, b):
    """mu1 and mu2 of one pair of angles by mpmath's tanh-sinh quadrature at 30 digits,
    on pieces of at most 6 rad of the faster oscillation."""
    import mpmath as mp
    with mp.workdps(30):
        a, b = mp.mpf(a), mp.mpf(b)
        sinc = lambda x: mp.sin(x) / x if x != 0 else mp.mpf(1)
        n = int(max(a, b) / 6) + 2
        pts = [mp.mpf(i) / n for i in range(n + 1)]
        m1 = -mp.quad(lambda t: t * t / 2 * mp.cos(t * a) * sinc(t * b / 2) ** 2, pts)
        m2 = mp.quad(lambda t: t * t * sinc(t * a) * sinc(t * b), pts)
    return float(m1), float(m2)


def test_pair_integrals_match_high_precision_quadrature_at_any_angle():
    """Rotation angles far beyond one turn (L-BFGS trial steps reach hundreds of rad):
    the oracle's composite rule against 30-digit quadrature, pairs of small, moderate and
    large angles in both orders."""
    sig = np.array([0.0, 0.3, 7.0, 45.0, 180.0, 450.0])
    mu1, mu2 = O.ov_pair_integrals(sig)
    pairs = [(0, 0), (1, 2), (2, 1), (3, 1), (1, 3), (4, 0), (0, 4), (3, 4), (4, 3), (5, 5),
             (5, 2), (2, 5), (5, 1)]
    for k, l in pairs:
        m1, m2 = _mp_pair_integrals(sig[k], sig[l])
        assert abs(mu1[k, l] - m1) < 1e-15, (sig[k], sig[l], mu1[k, l], m1)
        assert abs(mu2[k, l] - m2) < 1e-15, (sig[k], sig[l], mu2[k, l], m2)


def test_pair_integrals_closed_forms_at_large_angles():
    sig = np.array([1.0, 3.5, 41.0, 99.0, 230.0, 600.0])
    mu1, mu2 = O.ov_pair_integrals(sig)
    sk, sl = sig[:, None], sig[None, :]
    sincf = lambda x: np.sinc(x / np.pi)
    Kc = 0.5 * (sincf(sk - sl) + sincf(sk + sl))
    Ks = 0.5 * (sincf(sk - sl) - sincf(sk + sl))
    assert np.abs(mu1 - (Kc - sincf(sk)) / sl ** 2).max() < 1e-15
    assert np.abs(mu2 - Ks / (sk * sl)).max() < 1e-15


@pytest.mark.parametrize("M,N,scale", [(30, 6, 30.0), (12, 4, 100.0)])
def test_structured_ov_equals_dense_at_large_angles(M, N, scale):
    """sigma_max of about 200 and 380 rad: the structured path still equals the definition
    path.  Both lose accuracy as the angles grow (the eigendecompositions' errors scale with
    |A| and |A|^2), hence the looser bound than at small angles."""
    wl = tiny_real(M, N, seed=M + N, scale=scale)
    p = O.parity_params(wl)
    sig = np.sqrt(np.linalg.eigvalsh(p[0] @ p[0].T).clip(0.0))
    assert sig.max() > 150.0
    E, (g,) = O.energy_grad(wl, p)
    E2, (g2,) = O.energy_grad_ov_workload(wl, p)
    assert abs(E - E2) < 1e-12 * abs(E)
    assert np.abs(g - g2).max() < 1e-11 * np.abs(g).max()


@pytest.mark.parametrize("case", ["real", "complex"])
def test_density_matrix_properties(case):
    """rho = C F C^dagger: Hermitian, its eigenvalues are the occupations (C is unitary),
    its trace is the electron count, its diagonal is the site density of the energy, and
    E = Tr(rho H0) + (U/2) sum diag(rho)^2 equals the oracle's energy."""
    wl = tiny_real(11, 4, seed=21, scale=0.6) if case == "real" else tiny_complex(7, nk_side=2, kT=0.3)
    if case == "complex":
        wl.hubbard_U = 0.5
        wl.couple = False
    p = O.parity_params(wl)
    rhos = O.density_matrices(wl, p)
    E = 0.0
    for inst, rho in zip(wl.instances, rhos):
        assert np.abs(rho - rho.conj().T).max() < 1e-14
        ev = np.sort(np.linalg.eigvalsh(rho))
        assert np.abs(ev - np.sort(inst.f)).max() < 1e-13
        assert abs(np.trace(rho).real - inst.f.sum()) < 1e-13
        d = np.real(np.diag(rho))
        E += inst.weight * float(np.real(np.sum(rho.T * inst.h0_dense()))) + 0.5 * wl.hubbard_U * float((d ** 2).sum())
    assert abs(E - O.energy(wl, p)) < 1e-12 * abs(E)
    # at A = 0 the reference density
    z = O.zero_params(wl)
    for inst, rho in zip(wl.instances, O.density_matrices(wl, z)):
        assert np.abs(rho - (inst.C0 * inst.f) @ inst.C0.conj().T).max() < 1e-15


def test_density_matrix_of_one_rotation_by_hand():
    """M = 2, N = 1, f = (2, 0), C0 = I, B = [[theta]]: C = [[cos, sin], [-sin, cos]], so
    rho = 2 [[cos^2, -cos sin], [-cos sin, sin^2]]."""
    th = 0.7
    inst = Instance(M=2, N=1, f=np.array([2.0, 0.0]), C0=np.eye(2), A=np.array([[th]]), H0=np.eye(2))
    wl = Workload(0, "2-level", "real_ov", 0.0, False, [inst])
    (rho,) = O.density_matrices(wl, [np.array([[th]])])
    c, s_ = np.cos(th), np.sin(th)
    assert np.abs(rho - 2.0 * np.array([[c * c, -c * s_], [-c * s_, s_ * s_]])).max() < 1e-15


# ---------------------------------------------------------------------------
# minima
# ---------------------------------------------------------------------------

def test_minimum_without_interaction_is_ky_fan_sum():
    """U = 0: min E = sum_i f_i(desc) eps_i(asc) (von Neumann trace bound)."""
    wl = tiny_real(14, 4, seed=15)
    wl.hubbard_U = 0.0
    st, _ = LB.minimize(wl)
    ev = np.linalg.eigvalsh(wl.instances[0].H0)
    assert np.linalg.norm(st.g) < 1e-8
    assert abs(st.f - 2.0 * ev[:4].sum()) < 1e-10


def test_minimum_complex_fractional_occupations_ky_fan():
    wl = tiny_complex(8, nk_side=2, kT=0.3, hubbard_U=0.0)
    st, _ = LB.minimize(wl)
    ref = sum(i.weight * np.sort(i.f)[::-1] @ np.linalg.eigvalsh(i.H0) for i in wl.instances)
    assert np.linalg.norm(st.g) < 1e-8
    assert abs(st.f - ref) < 1e-10


def test_brute_force_minimum_three_levels():
    """M = 3, N = 1 with the Hubbard term: the occupied orbital is a point on S^2;
    a dense angular grid plus local polish gives the global minimum."""
    H0 = chain_hamiltonian(3, rng_for(300, 0, 0))
    Uh = 0.5

    def E_of(c):
        c = c / np.linalg.norm(c)
        return 2.0 * c @ H0 @ c + 0.5 * Uh * np.sum((2.0 * c * c) ** 2)
    best = None
    for th in np.linspace(0, np.pi, 181):
        for ph in np.linspace(0, 2 * np.pi, 361):
            c = np.array([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)])
            e = E_of(c)
            if best is None or e < best[0]:
                best = (e, c)
    res = scipy.optimize.minimize(E_of, best[1], method="BFGS", options=dict(gtol=1e-12))
    C0 = haar_orthogonal(3, rng_for(300, 0, 1))
    inst = Instance(M=3, N=1, f=np.array([2.0, 0.0, 0.0]), C0=C0, A=np.zeros((1, 2)), H0=H0)
    wl = Workload(300, "3-level", "real_ov", Uh, False, [inst])
    st, _ = LB.minimize(wl)
    assert abs(st.f - res.fun) < 1e-10


def test_brute_force_minimum_grassmannian_4_2():
    """M = 4, N = 2 with the Hubbard term: multistart over 2-frames in R^4."""
    H0 = chain_hamiltonian(4, rng_for(301, 0, 0))
    Uh = 0.5

    def E_of(x):
        Q, _ = np.linalg.qr(x.reshape(4, 2))
        rho = 2.0 * Q @ Q.T
        return np.sum(rho * H0) + 0.5 * Uh * np.sum(np.diag(rho) ** 2)
    rng = np.random.default_rng(0)
    best = min((scipy.optimize.minimize(E_of, rng.standard_normal(8), method="BFGS",
                                        options=dict(gtol=1e-12)).fun for _ in range(40)))
    C0 = haar_orthogonal(4, rng_for(301, 0, 1))
    inst = Instance(M=4, N=2, f=np.array([2.0, 2.0, 0.0, 0.0]), C0=C0, A=np.zeros((2, 2)), H0=H0)
    wl = Workload(301, "4-level", "real_ov", Uh, False, [inst])
    st, _ = LB.minimize(wl)
    assert abs(st.f - best) < 1e-10


def test_config1_lbfgs_reaches_scf_fixed_point():
    """Config 1: L-BFGS from A = 0 to |g| < 1e-8 lands on the Roothaan SCF fixed point."""
    wl = make_config(1)
    inst = wl.instances[0]
    rho0 = inst.C0 @ np.diag(inst.f) @ inst.C0.T
    E_scf, rho_scf, _ = scf.scf_minimum(inst.H0, inst.N, 2.0, wl.hubbard_U, rho0)
    st, hist = LB.minimize(wl)
    assert np.linalg.norm(st.g) < 1e-8
    assert abs(st.f - E_scf) < 1e-10
    B = O.unflatten("real_ov", wl, st.x)[0]
    C = wl.instances[0].C0 @ O.expm_eig(O.ov_generator(B))
    rho = 2.0 * C[:, :16] @ C[:, :16].T
    assert np.abs(rho - rho_scf).max() < 1e-7
    # energies never increase along accepted steps
    Es = [h["E"] for h in hist]
    assert all(b <= a + 1e-12 for a, b in zip(Es, Es[1:]))


def test_config1_lbfgs_with_norm_resets_reaches_scf_fixed_point():
    """Resets whenever |A| > 1 (the paper's norm rule, on top of every 20 iterations)
    keep |A| small and still reach the Roothaan SCF fixed point."""
    wl = make_config(1)
    inst = wl.instances[0]
    rho0 = inst.C0 @ np.diag(inst.f) @ inst.C0.T
    E_scf, _, _ = scf.scf_minimum(inst.H0, inst.N, 2.0, wl.hubbard_U, rho0)
    norms = []
    st, hist = LB.minimize(wl, reset_norm=1.0,
                           callback=lambda s, info: norms.append(np.linalg.norm(s.x)))
    assert np.linalg.norm(st.g) < 1e-8
    assert abs(st.f - E_scf) < 1e-10
    n_periodic = (len(hist) - 2) // 20
    assert hist[-1]["resets"] > n_periodic + 3
    # a reset follows every iterate above the threshold
    for k in range(len(norms) - 1):
        if norms[k] > 1.0:
            assert hist[k + 2]["resets"] == hist[k + 1]["resets"] + 1, k


def test_planted_mistakes_are_caught():
    """A dropped Hubbard term or a transposed gradient fails the finite-difference pin."""
    wl = tiny_real(9, 3, seed=16, scale=0.3)
    p = O.parity_params(wl)
    E, (g,) = O.energy_grad(wl, p)
    d = np.random.default_rng(2).standard_normal(g.size)
    fd = _fd_directional(wl, p, d, 1e-3)
    assert abs(fd - g.ravel() @ d) < 1e-8
    wl0 = copy.deepcopy(wl)
    wl0.hubbard_U = 0.0
    _, (g0,) = O.energy_grad(wl0, p)
    assert abs(fd - g0.ravel() @ d) > 1e-4
    # a mirrored index convention (g from Y_ij instead of Y_ji) flips the sign
    A, L, Y = O.y_matrix(wl, p, 0)
    g_bad = 2.0 * Y[:3, 3:]
    assert abs(fd - g_bad.ravel() @ d) > 1e-4
