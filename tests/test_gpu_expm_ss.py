"""exp(A) by scaling and squaring with a diagonal Pade approximant (Sec. 3.4, Eq. ss)
on the complex path, with the approximate gradient G ~ L^T of the paper's "ss"
configuration (against the oracle's expm_ss and energy_grad_approx(expm=expm_ss)) and
with the exact gradient through the Frechet derivative of exp (against the oracle's
energy_grad_ss and the eigenbasis gradient); and against the eigendecomposition path.  FP64 tolerances: energies 1e-12 relative,
gradients 1e-10 relative, unitaries 1e-13 absolute times 2^s for the s squarings (the
GPU scales to theta_9 and uses degree 9: up to two squarings more than the oracle's
degree-13 choice)."""
import numpy as np
import pytest

from oracle import etdm as O
from workloads import make_config, tiny_complex

from gpu_helpers import energy_grad, expm, make_handle, rel_err

pytestmark = pytest.mark.gpu


def _workload(which):
    if which == "tiny":
        return tiny_complex(12, nk_side=2, kT=0.3), 1.0
    if which == "odd":
        return tiny_complex(13, nk_side=1, kT=0.1), 1.0
    wl = make_config(4, nk=8)
    wl.instances = wl.instances[:8]
    return wl, (30.0 if which == "config4_8k_large" else 1.0)


@pytest.mark.parametrize("which", ["tiny", "odd", "config4_8k", "config4_8k_large"])
def test_ss_matches_oracle(which):
    wl, scale = _workload(which)
    params = [scale * p for p in O.parity_params(wl)]
    s_max = max(O.pade_degree_and_scaling(float(np.abs(O.generator(wl.kind, p)).sum(axis=0).max()))[1]
                for p in params)
    print(f"[case] ss {which} (oracle halvings up to {s_max})", flush=True)
    h, _ = make_handle(wl, "fp64", gradient="approx", expm="ss")
    E, G = energy_grad(h, wl, params)
    U = expm(h, wl, params)
    h.close()
    E_ref, G_ref = O.energy_grad_approx(wl, params, expm=O.expm_ss)
    assert abs(E[-1] - E_ref) <= 1e-12 * max(1.0, abs(E_ref))
    assert rel_err(G, G_ref) < 1e-10
    for u, p in zip(U, params):
        assert np.abs(u - O.expm_ss(O.generator(wl.kind, p))).max() < 1e-13 * 2.0 ** (s_max + 2)


def test_ss_equals_eigendecomposition_path():
    wl, _ = _workload("config4_8k")
    params = O.parity_params(wl)
    print("[case] ss vs eig, approximate gradient", flush=True)
    he, _ = make_handle(wl, "fp64", gradient="approx")
    hs, _ = make_handle(wl, "fp64", gradient="approx", expm="ss")
    Ee, Ge = energy_grad(he, wl, params)
    Es, Gs = energy_grad(hs, wl, params)
    he.close()
    hs.close()
    assert abs(Ee[-1] - Es[-1]) <= 1e-12 * abs(Ee[-1])
    assert rel_err(Gs, Ge) < 1e-10


def test_ss_zero_rotation_and_lbfgs():
    """A = 0: exp(A) = I exactly (no squarings, q(0) = p(0) = I).  Then L-BFGS
    iterations on the ss path (graphs requested, evaluations launched eagerly) lower E."""
    import torch
    wl = tiny_complex(8, nk_side=2, kT=0.3)
    print("[case] ss zero rotation and L-BFGS", flush=True)
    h, _ = make_handle(wl, "fp64", gradient="approx", expm="ss")
    U = expm(h, wl, O.zero_params(wl))
    for u in U:
        assert np.array_equal(u, np.eye(u.shape[0]))
    h.set_graph(True)
    A = torch.zeros(h.n_param, dtype=torch.float64, device="cuda:0")
    E = torch.empty(h.n_inst + 1, dtype=torch.float64, device="cuda:0")
    G = torch.empty_like(A)
    infos = [h.lbfgs_step(A, E, G) for _ in range(10)]
    h.close()
    assert infos[-1]["E"] < infos[0]["E"]
    assert all(b["E"] <= a["E"] + 1e-6 * abs(a["E"]) for a, b in zip(infos, infos[1:]))


@pytest.mark.parametrize("which", ["tiny", "odd", "config4_8k", "config4_8k_large"])
def test_ss_exact_gradient_matches_oracle(which):
    """Y = L(A, L) exp(A)^H with the Frechet derivative from the same scaling and squaring."""
    wl, scale = _workload(which)
    params = [scale * p for p in O.parity_params(wl)]
    print(f"[case] ss exact gradient {which}", flush=True)
    h, _ = make_handle(wl, "fp64", expm="ss")
    E, G = energy_grad(h, wl, params)
    h.close()
    E_ref, G_ref = O.energy_grad_ss(wl, params)
    assert abs(E[-1] - E_ref) <= 1e-12 * max(1.0, abs(E_ref))
    assert rel_err(G, G_ref) < 1e-10 * max(1.0, scale)
    E_eig, G_eig = O.energy_grad(wl, params)
    assert rel_err(G, G_eig) < 1e-10 * max(1.0, scale)


def test_ss_exact_lbfgs_steps():
    """L-BFGS with the exact gradient on the ss path: energies do not increase (beyond the
    approximate-Wolfe allowance) and every returned G is the oracle's exact gradient at
    the returned A.  (Whole trajectories of this case drift apart under rounding-level
    perturbations, so they are not compared with the eigendecomposition path's.)"""
    import torch
    from workloads.pack import unpack_params
    wl = tiny_complex(8, nk_side=2, kT=0.3)
    print("[case] ss exact L-BFGS", flush=True)
    h, _ = make_handle(wl, "fp64", expm="ss")
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


def _ragged_batch():
    """Three uncoupled instances of different M in one batch: M = 70 and 45 take three
    and two panels of the blocked solve (the last ones ragged) while M = 33 leaves off
    after its second panel of one row, and every panel spans several column groups."""
    parts = [tiny_complex(M, nk_side=1, kT=0.1, seed=s) for M, s in ((70, 1), (45, 2), (33, 3))]
    wl = parts[0]
    wl.instances = [p.instances[0] for p in parts]
    wl.couple = False
    wl.name = "ragged complex M = 70, 45, 33"
    return wl


@pytest.mark.parametrize("scale", [1.0, 20.0])
def test_ss_ragged_batch(scale):
    wl = _ragged_batch()
    params = [scale * p for p in O.parity_params(wl)]
    s_max = max(O.pade_degree_and_scaling(float(np.abs(O.generator(wl.kind, p)).sum(axis=0).max()))[1]
                for p in params)
    print(f"[case] ss ragged batch, scale {scale} (oracle halvings up to {s_max})", flush=True)
    h, _ = make_handle(wl, "fp64", gradient="approx", expm="ss")
    E, G = energy_grad(h, wl, params)
    U = expm(h, wl, params)
    h.close()
    E_ref, G_ref = O.energy_grad_approx(wl, params, expm=O.expm_ss)
    assert abs(E[-1] - E_ref) <= 1e-12 * max(1.0, abs(E_ref))
    assert rel_err(G, G_ref) < 1e-10
    for u, p in zip(U, params):
        assert np.abs(u - O.expm_ss(O.generator(wl.kind, p))).max() < 1e-13 * 2.0 ** (s_max + 2)
    h, _ = make_handle(wl, "fp64", expm="ss")
    E, G = energy_grad(h, wl, params)
    h.close()
    E_ref, G_ref = O.energy_grad_ss(wl, params)
    assert abs(E[-1] - E_ref) <= 1e-12 * max(1.0, abs(E_ref))
    assert rel_err(G, G_ref) < 1e-10 * max(1.0, scale)


def test_ss_largest_size():
    """M = 1024, the largest size of the path: 16 column tiles of the norm, 32 panels of the
    solve with 63 column groups each, and 16 x 16 tiles in every product; exp(A) and both
    gradients against the oracle (same tolerances: the oracle's degree-13 exponential and
    the eigenbasis agree to 3e-15 at this size)."""
    wl = tiny_complex(1024, nk_side=1, kT=0.1)
    params = O.parity_params(wl)
    s_max = max(O.pade_degree_and_scaling(float(np.abs(O.generator(wl.kind, p)).sum(axis=0).max()))[1]
                for p in params)
    print(f"[case] ss M = 1024 (oracle halvings up to {s_max})", flush=True)
    h, _ = make_handle(wl, "fp64", gradient="approx", expm="ss")
    E, G = energy_grad(h, wl, params)
    U = expm(h, wl, params)
    h.close()
    E_ref, G_ref = O.energy_grad_approx(wl, params, expm=O.expm_ss)
    assert abs(E[-1] - E_ref) <= 1e-12 * max(1.0, abs(E_ref))
    assert rel_err(G, G_ref) < 1e-10
    assert np.abs(U[0] - O.expm_ss(O.generator(wl.kind, params[0]))).max() < 1e-13 * 2.0 ** (s_max + 2)
    h, _ = make_handle(wl, "fp64", expm="ss")
    E, G = energy_grad(h, wl, params)
    h.close()
    E_ref, G_ref = O.energy_grad_ss(wl, params)
    assert abs(E[-1] - E_ref) <= 1e-12 * max(1.0, abs(E_ref))
    assert rel_err(G, G_ref) < 1e-10
