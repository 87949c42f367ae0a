"""Pins of the oracle's L-BFGS internals (Sec. 3.1-3.3) against their definitions.

Each piece is checked on its own, against something other than the oracle code:
the explicit BFGS inverse-Hessian update the two-loop recursion stands for, exact
minimizers of cubic polynomials, hand-computed preconditioners of Eq. prec_3 and
orbital energies, and the line-search acceptance tests of Eq. strw1, strw2, aprw
and aprw2 evaluated at every point the search returns.
"""
import copy

import numpy as np
import pytest

from oracle import etdm as O
from oracle import lbfgs as LB
from workloads import Instance, Workload, make_config, tiny_complex, tiny_real


# ---------------------------------------------------------------------------
# two-loop recursion (Sec. 3.1)
# ---------------------------------------------------------------------------

def _explicit_inverse_hessian(S, Y, Pdiag):
    """H_k from H_0 = diag(Pdiag) by the BFGS inverse update, oldest pair first:
    H <- (I - rho s y^T) H (I - rho y s^T) + rho s s^T, rho = 1 / (y.s)."""
    n = Pdiag.size
    H = np.diag(Pdiag)
    I = np.eye(n)
    for s, y in zip(S, Y):
        rho = 1.0 / (y @ s)
        H = (I - rho * np.outer(s, y)) @ H @ (I - rho * np.outer(y, s)) + rho * np.outer(s, s)
    return H


def _pairs(n, m, rng):
    # curvature pairs of a fixed SPD quadratic, so y.s > 0 for every pair
    Q = rng.standard_normal((n, n))
    A = Q @ Q.T + n * np.eye(n)
    S = [rng.standard_normal(n) for _ in range(m)]
    Y = [A @ s + 0.1 * rng.standard_normal(n) for s in S]
    for s, y in zip(S, Y):
        assert y @ s > 0.0
    return S, Y


@pytest.mark.parametrize("m", [0, 1, 2, 3])
def test_two_loop_equals_explicit_bfgs_inverse_update(m):
    rng = np.random.default_rng(40 + m)
    n = 9
    S, Y = _pairs(n, m, rng)
    Pdiag = rng.uniform(0.2, 3.0, n)
    g = rng.standard_normal(n)
    H = _explicit_inverse_hessian(S, Y, Pdiag)
    p = LB.two_loop(g, S, Y, Pdiag)
    assert np.abs(p + H @ g).max() < 1e-12 * np.abs(H @ g).max()


def test_two_loop_secant_condition():
    """The updated inverse Hessian maps the newest y onto the newest s."""
    rng = np.random.default_rng(44)
    S, Y = _pairs(11, 3, rng)
    Pdiag = rng.uniform(0.5, 2.0, 11)
    p = LB.two_loop(Y[-1], S, Y, Pdiag)
    assert np.abs(p + S[-1]).max() < 1e-12 * np.abs(S[-1]).max()


# ---------------------------------------------------------------------------
# cubic interpolation (Sec. 3.2)
# ---------------------------------------------------------------------------

def _cubic(c3, c2, c1, c0):
    f = lambda a: ((c3 * a + c2) * a + c1) * a + c0
    df = lambda a: (3.0 * c3 * a + 2.0 * c2) * a + c1
    return f, df


@pytest.mark.parametrize("coef,amin,ends", [
    # phi' = 3 (a - 1.3)(a + 0.4): local minimum at 1.3
    ((1.0, -1.35, -1.56, 7.0), 1.3, [(0.0, 2.0), (2.0, 0.5), (0.9, 3.0)]),
    # phi' = -3 (a - 0.5)(a - 2.5): local minimum at 0.5
    ((-1.0, 4.5, -3.75, 1.0), 0.5, [(0.0, 1.5), (1.2, 0.1), (0.3, 2.0)]),
    # a quadratic: phi' = 2 (a - 0.7)
    ((0.0, 1.0, -1.4, 0.0), 0.7, [(0.0, 1.0), (2.0, -1.0)]),
])
def test_cubic_minimizer_exact_on_cubics(coef, amin, ends):
    f, df = _cubic(*coef)
    for a, b in ends:
        x = LB.cubic_minimizer(a, f(a), df(a), b, f(b), df(b))
        assert x is not None and abs(x - amin) < 1e-12, (a, b, x)


def test_cubic_minimizer_none_without_a_minimizer():
    # phi' = 3 a^2 + 1 > 0 everywhere: no stationary point, so no minimizer
    f, df = _cubic(1.0, 0.0, 1.0, 0.0)
    assert LB.cubic_minimizer(-1.0, f(-1.0), df(-1.0), 1.0, f(1.0), df(1.0)) is None


# ---------------------------------------------------------------------------
# preconditioner (Sec. 3.3, Eq. prec_3) and orbital energies
# ---------------------------------------------------------------------------

def test_preconditioner_three_levels_by_hand():
    """M = 3, N = 1, f = (2, 0, 0), eps = (-1, 0.5, 2), gamma = 0.25, beta = 3:
    h_0j = -2 (eps_0 - eps_j)(f_0 - f_j) = 6 and 12, and
    P = 1 / ((1 - gamma) h + gamma beta) = 1 / 5.25 and 1 / 9.75."""
    inst = Instance(M=3, N=1, f=np.array([2.0, 0.0, 0.0]), C0=np.eye(3), A=np.zeros((1, 2)),
                    H0=np.eye(3))
    wl = Workload(0, "3-level", "real_ov", 0.0, False, [inst])
    h = LB.hessian_diagonal(wl, [np.array([-1.0, 0.5, 2.0])])
    assert np.array_equal(h, [6.0, 12.0])
    P = LB.preconditioner(h, LB.weight_vector(wl), 3.0, 0.25)
    assert np.abs(P - [1.0 / 5.25, 1.0 / 9.75]).max() < 1e-16


def test_preconditioner_clamps_wrong_order_and_keeps_beta_term():
    """An occupied level above a virtual one gives a negative Hessian term: clamped to 0,
    leaving P = 1 / (gamma beta)."""
    inst = Instance(M=3, N=1, f=np.array([2.0, 0.0, 0.0]), C0=np.eye(3), A=np.zeros((1, 2)),
                    H0=np.eye(3))
    wl = Workload(0, "3-level", "real_ov", 0.0, False, [inst])
    h = LB.hessian_diagonal(wl, [np.array([1.0, 0.5, 2.0])])
    assert np.array_equal(h, [0.0, 4.0])
    P = LB.preconditioner(h, LB.weight_vector(wl), 2.0, 0.25)
    assert np.abs(P - [1.0 / 0.5, 1.0 / 3.5]).max() < 1e-15


def test_preconditioner_complex_layout_and_weight_by_hand():
    """M = 2 complex k-point with weight 1/2, f = (1.5, 0.25), eps = (-0.5, 1.5):
    the free variables are Re a_01, Im a_00, Im a_01, Im a_11, and
    h_01 = w * (-2)(eps_0 - eps_1)(f_0 - f_1) = 0.5 * 5 = 2.5, h_ii = 0;
    P = 1 / ((1 - gamma) h + gamma beta w) with beta = 4, gamma = 0.25."""
    inst = Instance(M=2, N=2, f=np.array([1.5, 0.25]), C0=np.eye(2, dtype=complex),
                    A=np.zeros((2, 2), complex), H0=np.eye(2, dtype=complex), weight=0.5)
    wl = Workload(0, "2-level", "complex_full", 0.0, False, [inst])
    h = LB.hessian_diagonal(wl, [np.array([-0.5, 1.5])])
    assert np.array_equal(h, [2.5, 0.0, 2.5, 0.0])
    w = LB.weight_vector(wl)
    assert np.array_equal(w, [0.5] * 4)
    P = LB.preconditioner(h, w, 4.0, 0.25)
    assert np.abs(P - [1.0 / 2.375, 2.0, 1.0 / 2.375, 2.0]).max() < 1e-15


def test_orbital_energies_by_hand():
    """C0 = I, H0 = [[1, 0.2, 0], [0.2, 2, 0], [0, 0, 3]], f = (2, 0, 0), U = 0.5:
    n = diag(C0 F C0^T) = (2, 0, 0), H = H0 + U diag(n), eps = diag(H) = (2, 2, 3)."""
    H0 = np.array([[1.0, 0.2, 0.0], [0.2, 2.0, 0.0], [0.0, 0.0, 3.0]])
    inst = Instance(M=3, N=1, f=np.array([2.0, 0.0, 0.0]), C0=np.eye(3), A=np.zeros((1, 2)), H0=H0)
    wl = Workload(0, "3-level", "real_ov", 0.5, False, [inst])
    (eps,) = O.orbital_energies(wl)
    assert np.abs(eps - [2.0, 2.0, 3.0]).max() < 1e-15
    # a rotated reference: eps_i = c_i^T H c_i for its columns
    c = np.sqrt(0.5)
    C0 = np.array([[c, c, 0.0], [c, -c, 0.0], [0.0, 0.0, 1.0]])
    inst.C0 = C0
    (eps,) = O.orbital_energies(wl)
    # n = 2 (c0 * c0) = (1, 1, 0); H = H0 + 0.5 diag(1, 1, 0)
    H = H0 + 0.5 * np.diag([1.0, 1.0, 0.0])
    assert abs(eps[0] - (0.5 * (H[0, 0] + H[1, 1]) + H[0, 1])) < 1e-15
    assert abs(eps[1] - (0.5 * (H[0, 0] + H[1, 1]) - H[0, 1])) < 1e-15
    assert abs(eps[2] - 3.0) < 1e-15


# ---------------------------------------------------------------------------
# line search (Sec. 3.2): every returned point passes the acceptance tests
# ---------------------------------------------------------------------------

def _accepted(cfg, f0, d0, a, f, d):
    strong = f <= f0 + cfg.c1 * a * d0 and abs(d) <= cfg.c2 * abs(d0)
    approx = ((2.0 * cfg.delta - 1.0) * d0 >= d >= cfg.sigma * d0
              and f <= f0 + cfg.eps * abs(f0))
    return strong or approx


@pytest.mark.parametrize("case", ["config1", "tiny_real", "tiny_complex"])
def test_line_search_returns_only_wolfe_points(case, monkeypatch):
    """Every point the search accepts satisfies strong Wolfe (Eq. strw1, strw2), or
    approximate Wolfe (Eq. aprw) with the energy condition (Eq. aprw2); E and the slope
    there are recomputed from the definition path."""
    if case == "config1":
        wl, iters = make_config(1), 40
    elif case == "tiny_real":
        wl, iters = tiny_real(14, 4, seed=3), 30
    else:
        wl, iters = tiny_complex(6, nk_side=2, kT=0.2), 20
    cfg = LB.LbfgsConfig(max_iter=iters)
    real_ls = LB.line_search
    calls = []

    def recording(fun, x, f0, g0, p, c):
        res = real_ls(fun, x, f0, g0, p, c)
        calls.append((x.copy(), p.copy(), f0, float(g0 @ p), res))
        return res
    monkeypatch.setattr(LB, "line_search", recording)
    # no reference resets, so every x refers to the same reference orbitals
    LB.minimize(copy.deepcopy(wl), cfg, reset_every=0)
    kind = wl.kind
    n_checked = 0
    for x, p, f0, d0, res in calls:
        assert d0 < 0.0
        if not res.ok:
            continue
        E, gs = O.energy_grad(wl, O.unflatten(kind, wl, x + res.alpha * p))
        assert abs(E - res.f) <= 1e-12 * max(1.0, abs(E))
        d = float(O.flatten(kind, gs) @ p)
        assert _accepted(cfg, f0, d0, res.alpha, E, d), (res.alpha, f0, E, d0, d)
        n_checked += 1
    assert n_checked >= iters // 2
