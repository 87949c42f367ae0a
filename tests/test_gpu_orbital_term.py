"""The orbital-dependent model term (the PZ-SIC form of L, Sec. 2) on the complex path,
through the C ABI, against the oracle's energy_grad_odd (itself pinned by finite
differences): with exp(A) and Y through the eigendecomposition and through scaling
and squaring with the Frechet derivative.  FP64 tolerances: energies 1e-12 relative,
gradients 1e-10 relative."""
import numpy as np
import pytest

from oracle import etdm as O
from workloads import make_config, tiny_complex, with_overlap
from workloads.pack import unpack_params

from gpu_helpers import energy_grad, make_handle, rel_err

pytestmark = pytest.mark.gpu

LAM = 0.7


def _workload(which):
    if which == "tiny":
        return tiny_complex(12, nk_side=2, kT=0.3), 3.0
    if which == "tiny_overlap":  # Lowdin coefficients in the term, as in the site density
        return with_overlap(tiny_complex(12, nk_side=2, kT=0.3)), 2.0
    wl = make_config(4, nk=8)
    wl.instances = wl.instances[:8]
    return wl, 1.0


@pytest.mark.parametrize("which,expm", [("tiny", "eig"), ("tiny", "ss"), ("config4_8k", "eig"),
                                        ("config4_8k", "ss"), ("tiny_overlap", "eig"), ("tiny_overlap", "ss")])
def test_orbital_term_matches_oracle(which, expm):
    wl, scale = _workload(which)
    params = [scale * p for p in O.parity_params(wl)]
    print(f"[case] orbital-dependent term {which} {expm}", flush=True)
    h, _ = make_handle(wl, "fp64", expm=expm, odd_lambda=LAM)
    E, G = energy_grad(h, wl, params)
    h.close()
    E_ref, G_ref = O.energy_grad_odd(wl, params, LAM)
    assert abs(E[-1] - E_ref) <= 1e-12 * max(1.0, abs(E_ref))
    assert rel_err(G, G_ref) < 1e-10


def test_orbital_term_lbfgs_steps():
    """L-BFGS with the orbital-dependent term: energies do not increase beyond the
    approximate-Wolfe allowance and every returned G is the oracle's gradient at A."""
    import torch
    wl = tiny_complex(8, nk_side=2, kT=0.3)
    print("[case] orbital-dependent term L-BFGS", flush=True)
    h, _ = make_handle(wl, "fp64", odd_lambda=LAM)
    A = torch.zeros(h.n_param, dtype=torch.float64, device="cuda:0")
    E = torch.empty(h.n_inst + 1, dtype=torch.float64, device="cuda:0")
    G = torch.empty_like(A)
    prev = None
    for _ in range(6):
        info = h.lbfgs_step(A, E, G)
        params = unpack_params(wl, A.cpu().numpy())
        E_ref, G_ref = O.energy_grad_odd(wl, params, LAM)
        assert abs(info["E"] - E_ref) <= 1e-12 * max(1.0, abs(E_ref))
        assert rel_err(unpack_params(wl, G.cpu().numpy()), G_ref) < 1e-10
        if prev is not None:
            assert info["E"] <= prev + 1e-6 * abs(prev)
        prev = info["E"]
    h.close()


@pytest.mark.parametrize("which,expm", [("tiny", "eig"), ("tiny", "ss"), ("tiny_overlap", "eig"),
                                        ("tiny_overlap", "ss")])
def test_orbital_term_approx_gradient(which, expm):
    """G ~ L^T with the term's part in L, against the oracle's energy_grad_approx(lam=...)
    (equal to the exact gradient at A = 0, where the oracle pins it)."""
    wl, scale = _workload(which)
    params = [scale * p for p in O.parity_params(wl)]
    print(f"[case] orbital-dependent term, approximate gradient {which} {expm}", flush=True)
    h, _ = make_handle(wl, "fp64", gradient="approx", expm=expm, odd_lambda=LAM)
    E, G = energy_grad(h, wl, params)
    h.close()
    E_ref, G_ref = O.energy_grad_approx(wl, params, expm=O.expm_ss if expm == "ss" else None, lam=LAM)
    assert abs(E[-1] - E_ref) <= 1e-12 * max(1.0, abs(E_ref))
    assert rel_err(G, G_ref) < 1e-10
