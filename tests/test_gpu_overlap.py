"""A non-orthogonal basis (Sec. 2: C^H S C = I) through the C ABI: etdm_create applies
the Lowdin transform (Newton-Schulz for S^+-1/2 as grouped GEMMs) and the handle then
runs the orthonormal path.  Against the oracle, which works in the non-orthogonal basis
directly (Lowdin populations, H = H0 + U S^1/2 diag(n) S^1/2).  FP64 tolerances:
energies 1e-12 relative, gradients 1e-10 relative; mixed: |dE|/N_e < 1e-8, rel |dg| <
1e-6."""
import numpy as np
import pytest

from oracle import etdm as O
from workloads import make_config, tiny_complex, tiny_real, with_overlap

from gpu_helpers import energy_grad, make_handle, rel_err

pytestmark = pytest.mark.gpu


def _workload(which):
    if which == "real":
        return with_overlap(tiny_real(40, 8, seed=7, scale=0.3))
    if which == "config1":
        return with_overlap(make_config(1))
    return with_overlap(tiny_complex(12, nk_side=2, kT=0.3))


@pytest.mark.parametrize("which,precision,expm", [("real", "fp64", "eig"), ("config1", "fp64", "eig"),
                                                  ("config1", "mixed", "eig"), ("complex", "fp64", "eig"),
                                                  ("complex", "fp64", "ss")])
def test_overlap_matches_oracle(which, precision, expm):
    wl = _workload(which)
    params = O.parity_params(wl)
    print(f"[case] non-orthogonal basis {which} {precision} {expm}", flush=True)
    h, _ = make_handle(wl, precision, expm=expm)
    E, G = energy_grad(h, wl, params)
    h.close()
    E_ref, G_ref = O.energy_grad(wl, params)
    if precision == "fp64":
        assert abs(E[-1] - E_ref) <= 1e-12 * max(1.0, abs(E_ref))
        assert rel_err(G, G_ref) < 1e-10
    else:
        assert abs(E[-1] - E_ref) / wl.n_electrons < 1e-8
        assert rel_err(G, G_ref) < 1e-6


def test_overlap_not_positive_definite_is_rejected():
    from paper_2101_12597_amd import EtdmError
    wl = _workload("real")
    inst = wl.instances[0]
    inst.S = inst.S - 2.0 * np.eye(inst.M)  # indefinite
    print("[case] indefinite overlap", flush=True)
    with pytest.raises(EtdmError) as e:
        make_handle(wl, "fp64")
    assert e.value.code == -1


@pytest.mark.parametrize("which,expm", [("real", "eig"), ("config1", "eig"), ("complex", "eig"), ("complex", "ss")])
def test_overlap_approx_gradient_matches_oracle(which, expm):
    """The approximate gradient G ~ L^T in a non-orthogonal basis, against the oracle's
    energy_grad_approx (Lowdin site densities)."""
    wl = _workload(which)
    params = O.parity_params(wl)
    print(f"[case] non-orthogonal basis, approximate gradient {which} {expm}", flush=True)
    h, _ = make_handle(wl, "fp64", gradient="approx", expm=expm)
    E, G = energy_grad(h, wl, params)
    h.close()
    E_ref, G_ref = O.energy_grad_approx(wl, params, expm=O.expm_ss if expm == "ss" else None)
    assert abs(E[-1] - E_ref) <= 1e-12 * max(1.0, abs(E_ref))
    assert rel_err(G, G_ref) < 1e-10


@pytest.mark.parametrize("which", ["real", "complex"])
def test_overlap_lbfgs_steps(which):
    """L-BFGS on a handle with an overlap: energies do not increase (beyond the
    approximate-Wolfe allowance), and E and G at every returned A are the oracle's in the
    non-orthogonal basis (no reference reset within these steps, so the reference is the
    caller's C0)."""
    import torch
    from workloads.pack import unpack_params
    wl = _workload(which)
    print(f"[case] non-orthogonal basis, L-BFGS {which}", flush=True)
    h, _ = make_handle(wl, "fp64")
    A = torch.zeros(h.n_param, dtype=torch.float64, device="cuda:0")
    E = torch.empty(h.n_inst + 1, dtype=torch.float64, device="cuda:0")
    G = torch.empty_like(A)
    prev = None
    for _ in range(6):
        info = h.lbfgs_step(A, E, G)
        assert not info["flags"] & 1
        params = unpack_params(wl, A.cpu().numpy())
        E_ref, G_ref = O.energy_grad(wl, params)
        assert abs(info["E"] - E_ref) <= 1e-12 * max(1.0, abs(E_ref))
        assert rel_err(unpack_params(wl, G.cpu().numpy()), G_ref) < 1e-10
        if prev is not None:
            assert info["E"] <= prev + 1e-6 * abs(prev)
        prev = info["E"]
    h.close()
