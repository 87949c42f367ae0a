"""The approximate gradient G ~ L^T (Sec. 3.4, Eq. app_grad) of the HIP path,
through the C ABI, against the oracle's energy_grad_approx (itself pinned to the
exact gradient at A = 0 and to its error order in A).

Tolerances as for the exact gradient: FP64 mode 1e-12 relative on energies and
1e-10 relative on gradients; mixed mode |dE| / N_e < 1e-8 Ha and
||dg|| / ||g|| < 1e-6 per instance.
"""
import copy

import numpy as np
import pytest

from oracle import etdm as O
from workloads import make_config, tiny_complex

from gpu_helpers import energy_grad, make_handle, rel_err
from test_gpu_parity import per_instance_errors, ragged_workload

pytestmark = pytest.mark.gpu


def _workload(which):
    if which == "config1":
        return make_config(1)
    if which == "ragged":
        return ragged_workload()
    if which == "config2":
        return make_config(2)
    if which == "config3":
        return make_config(3)
    if which == "tiny_complex":
        wl = tiny_complex(12, nk_side=2, kT=0.3)
        for inst in wl.instances:
            inst.A = inst.A * 6.0
        return wl
    wl = make_config(4, nk=8)
    wl.instances = wl.instances[:8]
    return wl


def _oracle_per_instance(wl, params):
    E_list, g_list = [], []
    for k, inst in enumerate(wl.instances):
        sub = copy.copy(wl)
        sub.instances = [inst]
        E, (g,) = O.energy_grad_approx(sub, [params[k]])
        E_list.append(E)
        g_list.append(g)
    return np.array(E_list), g_list


@pytest.mark.parametrize("which,precision", [("config1", "fp64"), ("ragged", "fp64"), ("ragged", "mixed"),
                                             ("config2", "mixed"), ("config3", "mixed")])
def test_real_ov_approx_matches_oracle(which, precision):
    wl = _workload(which)
    params = O.parity_params(wl)
    print(f"[case] approx gradient real_ov {which} {precision}", flush=True)
    h, _ = make_handle(wl, precision, use_bsr=which == "config3", gradient="approx")
    E, g = energy_grad(h, wl, params)
    h.close()
    E_ref, g_ref = _oracle_per_instance(wl, params)
    if precision == "fp64":
        for k in range(len(wl.instances)):
            assert abs(E[k] - E_ref[k]) <= 1e-12 * max(1.0, abs(E_ref[k])), k
        assert rel_err(g, g_ref) < 1e-10
    else:
        errs = per_instance_errors(wl, E, g, E_ref, g_ref)
        worst = max(e[0] for e in errs), max(e[1] for e in errs)
        print(f"[result] approx {which} mixed: max |dE|/Ne = {worst[0]:.3e}, max rel |dg| = {worst[1]:.3e}")
        assert worst[0] < 1e-8 and worst[1] < 1e-6


@pytest.mark.parametrize("which", ["tiny_complex", "config4_8k"])
def test_complex_approx_matches_oracle(which):
    wl = _workload(which)
    params = O.parity_params(wl)
    print(f"[case] approx gradient complex_full {which}", flush=True)
    h, _ = make_handle(wl, "fp64", gradient="approx")
    E, G = energy_grad(h, wl, params)
    h.close()
    E_ref, G_ref = O.energy_grad_approx(wl, params)
    assert abs(E[-1] - E_ref) <= 1e-12 * max(1.0, abs(E_ref))
    assert rel_err(G, G_ref) < 1e-10


@pytest.mark.parametrize("which", ["ragged", "tiny_complex"])
def test_approx_equals_exact_at_zero(which):
    """At A = 0 every divided-difference factor is 1, so Y = L and both modes agree."""
    wl = _workload(which)
    params = [np.zeros_like(p) for p in O.parity_params(wl)]
    print(f"[case] approx vs exact at A = 0 {which}", flush=True)
    he, _ = make_handle(wl, "fp64")
    ha, _ = make_handle(wl, "fp64", gradient="approx")
    Ee, ge = energy_grad(he, wl, params)
    Ea, ga = energy_grad(ha, wl, params)
    he.close()
    ha.close()
    assert np.array_equal(Ee, Ea)
    assert rel_err(ga, ge) < 1e-12


def test_approx_graph_replay_matches_eager():
    import torch
    wl = make_config(2)
    params = O.parity_params(wl)
    print("[case] approx gradient graph replay config2 mixed", flush=True)
    h, _ = make_handle(wl, "mixed", gradient="approx")
    ref = energy_grad(h, wl, params)
    h.set_graph(True)
    for rep in range(3):
        E, g = energy_grad(h, wl, params)
        assert np.array_equal(E, ref[0]), rep
        assert all(np.array_equal(a, b) for a, b in zip(g, ref[1])), rep
        torch.cuda.synchronize()
    h.close()
