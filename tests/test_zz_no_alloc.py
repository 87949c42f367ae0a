"""The allocation-free entry point etdm_energy_grad_static against etdm_energy_grad (a
handle, FP64) on the same inputs: two calls in a row, the second on a smaller
instance, then the same call replayed from a captured HIP graph.

Both run the same kernels in FP64 (the handle may pick other GEMM kernels for its
larger problems), so the bounds are those of the FP64 parity tests: E to 1e-12
relative, G to 1e-10 of its largest entry.
"""
import numpy as np
import pytest

from oracle import etdm as O
from workloads import make_config, tiny_real
from workloads.pack import pack

from gpu_helpers import energy_grad, make_handle

pytestmark = pytest.mark.gpu


def _static_call(wl, params, stream=None):
    import torch
    from paper_2101_12597_amd import energy_grad_static
    inst = wl.instances[0]
    M, N = inst.M, inst.N
    dev = torch.device("cuda:0")
    H0 = torch.from_numpy(np.ascontiguousarray(inst.H0)).to(dev)
    C0 = torch.from_numpy(np.ascontiguousarray(inst.C0)).to(dev)
    B = torch.from_numpy(np.ascontiguousarray(params[0])).to(dev)
    E = torch.full((2,), float("nan"), dtype=torch.float64, device=dev)
    G = torch.full((N * (M - N),), float("nan"), dtype=torch.float64, device=dev)
    st = torch.full((1,), -1, dtype=torch.int32, device=dev)
    return (M, N, float(inst.f[0]), wl.hubbard_U, H0, C0, B.reshape(-1), E, G, st), energy_grad_static


def _compare(wl, params, E, G, st):
    h, _ = make_handle(wl, "fp64")
    E_ref, (g_ref,) = energy_grad(h, wl, params)
    h.close()
    assert int(st.item()) == 0
    e = E.cpu().numpy()
    g = G.cpu().numpy().reshape(g_ref.shape)
    assert abs(e[0] - E_ref[0]) <= 1e-12 * abs(E_ref[0]) and abs(e[1] - E_ref[-1]) <= 1e-12 * abs(E_ref[-1])
    assert np.abs(g - g_ref).max() <= 1e-10 * np.abs(g_ref).max()
    # and the oracle's definition path
    E_o, (g_o,) = O.energy_grad(wl, params)
    assert abs(e[1] - E_o) <= 1e-12 * abs(E_o)
    assert np.abs(g - g_o).max() <= 1e-10 * np.abs(g_o).max()


def test_static_entry_point_matches_handle_two_calls():
    import torch
    big = tiny_real(200, 40, seed=31, scale=0.3)
    small = make_config(1)
    print("[case] static entry point M=200 N=40 then M=64 N=16", flush=True)
    for wl in (big, small):
        params = O.parity_params(wl)
        args, fn = _static_call(wl, params)
        fn(*args)
        torch.cuda.synchronize()
        _compare(wl, params, args[7], args[8], args[9])


def test_static_entry_point_rejects_sizes_beyond_its_array():
    import torch
    from paper_2101_12597_amd import EtdmError, energy_grad_static
    dev = torch.device("cuda:0")
    M, N = 401, 40
    z = lambda n, dt=torch.float64: torch.zeros(n, dtype=dt, device=dev)
    with pytest.raises(EtdmError):
        energy_grad_static(M, N, 2.0, 0.5, z(M * M), z(M * M), z(N * (M - N)), z(2), z(N * (M - N)),
                           z(1, torch.int32))
    M, N = 200, 89
    with pytest.raises(EtdmError):
        energy_grad_static(M, N, 2.0, 0.5, z(M * M), z(M * M), z(N * (M - N)), z(2), z(N * (M - N)),
                           z(1, torch.int32))


def test_static_entry_point_replays_from_a_captured_graph():
    """Captured once, replayed three times with eager work and other inputs between the
    replays; every replay equals the eager result bitwise."""
    import torch
    wl = tiny_real(120, 30, seed=32, scale=0.3)
    params = O.parity_params(wl)
    args, fn = _static_call(wl, params)
    print("[case] static entry point under graph capture", flush=True)
    fn(*args)
    torch.cuda.synchronize()
    E0, G0 = args[7].clone(), args[8].clone()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        fn(*args, stream=s)  # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=s):
        fn(*args, stream=s)
    for rep in range(3):
        args[7].fill_(float("nan"))
        args[8].fill_(float("nan"))
        # eager work and a call on other inputs in between
        other = tiny_real(64, 16, seed=33, scale=0.2)
        oargs, _ = _static_call(other, O.parity_params(other))
        fn(*oargs)
        x = torch.randn(1 << 18, device="cuda:0", dtype=torch.float64)
        assert torch.isfinite(x.sum()).item()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(args[7], E0) and torch.equal(args[8], G0), rep
        assert int(args[9].item()) == 0
