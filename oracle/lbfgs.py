"""Reference L-BFGS minimizer of E(A) (test infrastructure only).

Follows Sec. 3.1-3.3 of the paper:
  * search direction: L-BFGS two-loop recursion with m = 3 stored pairs, the
    diagonal preconditioner of Eq. prec_3 as the initial inverse Hessian;
  * step length: trial alpha = 1, accepted if the strong Wolfe conditions
    (Eq. strw1, strw2) hold; otherwise cubic interpolation of E along p using
    E and dE/dalpha at the ends of the search interval, accepting a point that
    satisfies strong Wolfe, or approximate Wolfe (Eq. aprw) together with the
    energy condition (Eq. aprw2);
  * constants c1 = 1e-4, c2 = 0.9, delta = 0.1, sigma = 0.9, eps = 1e-6, gamma = 0.25.

Readings where the paper is silent:
  * bracketing/zoom follow the usual expand-then-zoom scheme: expand while the
    slope stays negative and E keeps decreasing, zoom with safeguarded cubic
    steps (kept 10% away from the ends of the interval, bisection when the
    cubic has no minimizer);
  * beta^(0) = 1 Ha; beta keeps its previous value when s.y <= 0, and the pair
    is then not stored;
  * the Hessian term -2 (e_i - e_j)(f_i - f_j) is clamped at 0 so the
    preconditioner stays positive when C0 is not an eigenbasis; both terms are
    multiplied by the k-point weight (the paper's occupation numbers include it);
  * if p is not a descent direction, or the line search fails, the memory is
    erased and one preconditioned steepest-descent step is taken.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, List, Optional, Tuple

import numpy as np

from . import etdm


@dataclass
class LbfgsConfig:
    m: int = 3
    c1: float = 1e-4
    c2: float = 0.9
    delta: float = 0.1
    sigma: float = 0.9
    eps: float = 1e-6
    gamma: float = 0.25
    beta0: float = 1.0
    max_iter: int = 333
    max_ls: int = 20
    gtol: float = 1e-8


def hessian_diagonal(wl, eps_list) -> np.ndarray:
    """Flat vector of w_k * max(0, -2 (e_i - e_j)(f_i - f_j)) over the free variables."""
    parts = []
    for inst, e in zip(wl.instances, eps_list):
        f = inst.f
        h = -2.0 * (e[:, None] - e[None, :]) * (f[:, None] - f[None, :])
        h = inst.weight * np.maximum(h, 0.0)
        if wl.kind == "real_ov":
            N = inst.N
            parts.append(h[:N, N:].ravel())
        else:
            M = inst.M
            parts.append(h[np.triu_indices(M, 1)])
            parts.append(h[np.triu_indices(M, 0)])
    return np.concatenate(parts)


def weight_vector(wl) -> np.ndarray:
    parts = []
    for inst in wl.instances:
        M, N = inst.M, inst.N
        n = N * (M - N) if wl.kind == "real_ov" else M * M
        parts.append(np.full(n, inst.weight))
    return np.concatenate(parts)


def preconditioner(hdiag, wvec, beta, gamma) -> np.ndarray:
    """Eq. prec_3: P = 1 / ((1 - gamma) h + gamma beta w)."""
    return 1.0 / ((1.0 - gamma) * hdiag + gamma * beta * wvec)


def two_loop(g, S, Y, Pdiag) -> np.ndarray:
    """-H g by the L-BFGS two-loop recursion with H0 = diag(Pdiag)."""
    q = g.copy()
    alphas = []
    for s, y in reversed(list(zip(S, Y))):
        rho = 1.0 / np.dot(y, s)
        a = rho * np.dot(s, q)
        q -= a * y
        alphas.append((rho, a))
    r = Pdiag * q
    for (s, y), (rho, a) in zip(zip(S, Y), reversed(alphas)):
        b = rho * np.dot(y, r)
        r += s * (a - b)
    return -r


def cubic_minimizer(a, fa, ga, b, fb, gb) -> Optional[float]:
    """Minimizer of the cubic through (a, fa, fa') and (b, fb, fb'), or None."""
    if a == b:
        return None
    d1 = ga + gb - 3.0 * (fa - fb) / (a - b)
    disc = d1 * d1 - ga * gb
    if disc < 0.0:
        return None
    d2 = np.copysign(np.sqrt(disc), b - a)
    den = gb - ga + 2.0 * d2
    if den == 0.0:
        return None
    return b - (b - a) * (gb + d2 - d1) / den


@dataclass
class LineSearchResult:
    alpha: float
    f: float
    g: np.ndarray
    n_evals: int
    ok: bool


def line_search(fun: Callable, x, f0, g0, p, cfg: LbfgsConfig) -> LineSearchResult:
    dphi0 = float(np.dot(g0, p))
    n = 0

    def phi(a):
        nonlocal n
        n += 1
        f, g = fun(x + a * p)
        return f, g, float(np.dot(g, p))

    def strong_wolfe(a, f, d):
        return f <= f0 + cfg.c1 * a * dphi0 and abs(d) <= cfg.c2 * abs(dphi0)

    def approx_wolfe(f, d):
        return ((2.0 * cfg.delta - 1.0) * dphi0 >= d >= cfg.sigma * dphi0
                and f <= f0 + cfg.eps * abs(f0))

    best = (0.0, f0, g0)

    def note(a, f, g):
        nonlocal best
        if f < best[1]:
            best = (a, f, g)

    def zoom(lo, flo, dlo, hi, fhi, dhi):
        while n < cfg.max_ls:
            a = cubic_minimizer(lo, flo, dlo, hi, fhi, dhi)
            width = hi - lo
            left, right = min(lo, hi) + 0.1 * abs(width), max(lo, hi) - 0.1 * abs(width)
            if a is None or not np.isfinite(a) or a < left or a > right:
                a = 0.5 * (lo + hi)
            f, g, d = phi(a)
            note(a, f, g)
            if strong_wolfe(a, f, d) or approx_wolfe(f, d):
                return LineSearchResult(a, f, g, n, True)
            if f > f0 + cfg.c1 * a * dphi0 or f >= flo:
                hi, fhi, dhi = a, f, d
            else:
                if d * (hi - lo) >= 0.0:
                    hi, fhi, dhi = lo, flo, dlo
                lo, flo, dlo = a, f, d
        return None

    a_prev, f_prev, d_prev = 0.0, f0, dphi0
    a = 1.0
    f, g, d = phi(a)
    note(a, f, g)
    if strong_wolfe(a, f, d):
        return LineSearchResult(a, f, g, n, True)
    first = True
    while True:
        if f > f0 + cfg.c1 * a * dphi0 or (not first and f >= f_prev):
            res = zoom(a_prev, f_prev, d_prev, a, f, d)
            break
        if d >= 0.0:
            res = zoom(a, f, d, a_prev, f_prev, d_prev)
            break
        # still descending: extrapolate with the cubic, kept within [1.1 a, 4 a]
        a_new = cubic_minimizer(a_prev, f_prev, d_prev, a, f, d)
        if a_new is None or not np.isfinite(a_new) or a_new < 1.1 * a or a_new > 4.0 * a:
            a_new = 4.0 * a if (a_new is None or not np.isfinite(a_new) or a_new > 4.0 * a) else 1.1 * a
        a_prev, f_prev, d_prev = a, f, d
        if n >= cfg.max_ls:
            res = None
            break
        a = a_new
        f, g, d = phi(a)
        note(a, f, g)
        first = False
        if strong_wolfe(a, f, d) or approx_wolfe(f, d):
            return LineSearchResult(a, f, g, n, True)
    if res is not None:
        return res
    a, fb, gb = best
    return LineSearchResult(a, fb, gb, n, a > 0.0)


@dataclass
class LbfgsState:
    x: np.ndarray
    f: float
    g: np.ndarray
    beta: float
    S: List[np.ndarray] = field(default_factory=list)
    Y: List[np.ndarray] = field(default_factory=list)
    n_evals: int = 1
    n_iter: int = 0


def lbfgs_step(fun, st: LbfgsState, hdiag, wvec, cfg: LbfgsConfig) -> Tuple[LbfgsState, dict]:
    """One L-BFGS iteration (direction, line search, memory and beta update)."""
    P = preconditioner(hdiag, wvec, st.beta, cfg.gamma)
    p = two_loop(st.g, st.S, st.Y, P)
    fallback = False
    if not np.dot(p, st.g) < 0.0:
        st.S, st.Y = [], []
        p = -P * st.g
        fallback = True
    ls = line_search(fun, st.x, st.f, st.g, p, cfg)
    st.n_evals += ls.n_evals
    if not ls.ok:
        st.S, st.Y = [], []
        p = -P * st.g
        ls = line_search(fun, st.x, st.f, st.g, p, cfg)
        st.n_evals += ls.n_evals
        fallback = True
        if not ls.ok:
            return st, dict(alpha=0.0, failed=True, fallback=True)
    s = ls.alpha * p
    y = ls.g - st.g
    sy = float(np.dot(s, y))
    if sy > 0.0:
        st.S.append(s)
        st.Y.append(y)
        if len(st.S) > cfg.m:
            st.S.pop(0)
            st.Y.pop(0)
        st.beta = float(np.dot(y, y)) / sy
    st.x = st.x + s
    st.f = ls.f
    st.g = ls.g
    st.n_iter += 1
    return st, dict(alpha=ls.alpha, failed=False, fallback=fallback, evals=ls.n_evals)


def minimize(wl, cfg: Optional[LbfgsConfig] = None, reset_every: int = 20, callback=None,
             reset_norm: float = 0.0):
    """Minimize E from A = 0 with periodic reference-orbital resets (Sec. 3.4).

    Every ``reset_every`` iterations the reference orbitals are replaced by the
    current ones, C0 <- C0 exp(A), A <- 0, and the L-BFGS memory is erased (the
    paper's choice).  With ``reset_norm`` > 0 a reset also happens before an
    iteration whenever some instance's parameters have a 2-norm above it (the
    paper's suggestion to reset once the norm of A exceeds 1).  Reading: the orbital energies of the preconditioner are
    recomputed from the new reference orbitals ("at the beginning" of each
    cycle) and beta carries over.  ``wl`` is modified in place (its C0).
    Returns (final state, history); the final state's x refers to the last
    reference orbitals.
    """
    cfg = cfg or LbfgsConfig()
    kind = wl.kind

    def fun(v):
        E, gs = etdm.energy_grad(wl, etdm.unflatten(kind, wl, v))
        return E, etdm.flatten(kind, gs)

    wvec = weight_vector(wl)
    x = etdm.flatten(kind, etdm.zero_params(wl))
    f, g = fun(x)
    st = LbfgsState(x=x, f=f, g=g, beta=cfg.beta0)
    hdiag = hessian_diagonal(wl, etdm.orbital_energies(wl))
    history = [dict(E=f, gnorm=float(np.linalg.norm(g)), alpha=0.0, evals=1)]
    total_evals = 1
    total_iter = 0
    resets = 0
    while np.linalg.norm(st.g) >= cfg.gtol and total_iter < cfg.max_iter:
        periodic = reset_every and total_iter > 0 and total_iter % reset_every == 0
        large = reset_norm > 0.0 and max(np.linalg.norm(a) for a in etdm.unflatten(kind, wl, st.x)) > reset_norm
        if periodic or large:
            resets += 1
            reset_reference(wl, etdm.unflatten(kind, wl, st.x))
            x = etdm.flatten(kind, etdm.zero_params(wl))
            f, g = fun(x)
            total_evals += 1
            st = LbfgsState(x=x, f=f, g=g, beta=st.beta, n_iter=st.n_iter)
            hdiag = hessian_diagonal(wl, etdm.orbital_energies(wl))
        n_before = st.n_evals
        st, info = lbfgs_step(fun, st, hdiag, wvec, cfg)
        total_evals += st.n_evals - n_before
        total_iter += 1
        history.append(dict(E=st.f, gnorm=float(np.linalg.norm(st.g)), alpha=info["alpha"],
                            evals=total_evals, resets=resets))
        if callback:
            callback(st, info)
        if info["failed"]:
            break
    st.n_evals = total_evals
    st.n_iter = total_iter
    return st, history


def reset_reference(wl, params) -> None:
    """C0 <- C0 exp(A) for every instance (Sec. 3.4, update of the reference orbitals)."""
    for inst, a in zip(wl.instances, params):
        inst.C0 = inst.C0 @ etdm.expm_eig(etdm.generator(wl.kind, a))


def _complex_weight_vector(wl) -> np.ndarray:
    parts = []
    for inst in wl.instances:
        M = inst.M
        parts.append(np.full(M * (M - 1) // 2, inst.weight))
        parts.append(np.full(M * (M + 1) // 2, inst.weight))
    return np.concatenate(parts)
