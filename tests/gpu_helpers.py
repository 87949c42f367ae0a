"""Helpers shared by the GPU tests: build a library handle from a workload and
run the C-ABI entry points on device tensors."""
from __future__ import annotations

import numpy as np

from workloads.pack import pack, pack_params, unpack_params, unpack_square


def torch_dev():
    import torch
    return torch, torch.device("cuda:0")


def make_handle(wl, precision="fp64", use_bsr=False, gemm_tuning=0, gradient="exact", expm="eig",
                odd_lambda=0.0, want_rho=False):
    torch, dev = torch_dev()
    from paper_2101_12597_amd import Handle
    pk = pack(wl, use_bsr=use_bsr)
    H0 = torch.from_numpy(pk["H0"]).to(dev)
    C0 = torch.from_numpy(pk["C0"]).to(dev)
    S = torch.from_numpy(pk["S"]).to(dev) if pk.get("S") is not None else None
    h = Handle(pk["M"], pk["N"], wl.kind, precision, wl.hubbard_U, H0, C0, pk["f"],
               couple=wl.couple, weights=pk["weights"], bsr=pk["bsr"], gemm_tuning=gemm_tuning,
               gradient=gradient, expm=expm, odd_lambda=odd_lambda, overlap=S, want_rho=want_rho)
    torch.cuda.synchronize()
    return h, pk


def energy_grad(h, wl, params):
    torch, dev = torch_dev()
    A = torch.from_numpy(pack_params(wl, params)).to(dev)
    E = torch.empty(h.n_inst + 1, dtype=torch.float64, device=dev)
    G = torch.empty_like(A)
    h.energy_grad(A, E, G)
    h.sync_status()
    return E.cpu().numpy(), unpack_params(wl, G.cpu().numpy())


def expm(h, wl, params):
    torch, dev = torch_dev()
    A = torch.from_numpy(pack_params(wl, params)).to(dev)
    n = sum(2 * i.M * i.M if wl.kind != "real_ov" else i.M * i.M for i in wl.instances)
    U = torch.empty(n, dtype=torch.float64, device=dev)
    h.expm(A, U)
    h.sync_status()
    return unpack_square(wl, U.cpu().numpy())


def density(h, wl, params):
    """rho = C F C^dagger per instance through etdm_density, as host arrays."""
    torch, dev = torch_dev()
    A = torch.from_numpy(pack_params(wl, params)).to(dev)
    cplx = wl.kind != "real_ov"
    n = sum((2 if cplx else 1) * i.M * i.M for i in wl.instances)
    rho = torch.empty(n, dtype=torch.float64, device=dev)
    h.density(A, rho)
    h.sync_status()
    return unpack_square(wl, rho.cpu().numpy())


def rel_err(a, b):
    a = np.concatenate([np.ravel(x) for x in a])
    b = np.concatenate([np.ravel(x) for x in b])
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
