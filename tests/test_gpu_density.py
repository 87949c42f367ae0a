"""The full density matrix rho = C F C^dagger (etdm_density) against the oracle's
definition (C = C0 exp(A) from the eigendecomposition of iA), element by element.

Real instances: a symmetric rank-N product over row panels of the upper triangle,
then mirrored, in the precision of the contractions E depends on.  Bounds: FP64
1e-12 of max |rho|; split precision 2e-6 of max |rho| (the BF16x6 products carry about
1e-7 of the sum of the magnitudes of their terms, and |C_occ| rows have norm <= 1).
"""
import numpy as np
import pytest

from oracle import etdm as O
from workloads import make_config

from gpu_helpers import density, make_handle

pytestmark = pytest.mark.gpu

from test_gpu_parity import ragged_workload  # noqa: E402


@pytest.mark.parametrize("which,precision,tol", [("config1", "fp64", 1e-12), ("ragged", "fp64", 1e-12),
                                                 ("ragged", "bf16x6", 2e-6), ("config3", "mixed", 1e-12),
                                                 ("config3", "bf16x6", 2e-6), ("config4_8k", "fp64", 1e-12)])
def test_density_matches_oracle(which, precision, tol):
    if which == "config1":
        wl = make_config(1)
    elif which == "ragged":
        wl = ragged_workload()
    elif which == "config3":
        wl = make_config(3)
    else:
        wl = make_config(4, nk=8)
        wl.instances = wl.instances[:8]
    params = O.parity_params(wl)
    print(f"[case] density {which} {precision}", flush=True)
    h, _ = make_handle(wl, precision, use_bsr=which == "config3", want_rho=True)
    rho = density(h, wl, params)
    h.close()
    ref = O.density_matrices(wl, params)
    worst = 0.0
    for k, (r, q) in enumerate(zip(rho, ref)):
        scale = max(np.abs(q).max(), 1e-300)
        err = np.abs(r - q).max() / scale
        worst = max(worst, err)
        assert err < tol, (k, wl.instances[k].M, wl.instances[k].N, err)
        # exactly symmetric / Hermitian: the lower triangle is the mirrored upper one
        assert np.array_equal(r, r.conj().T), k
    print(f"[result] density {which} {precision}: max |d rho| / max |rho| = {worst:.3e}")


def test_density_requires_want_rho():
    import torch
    from paper_2101_12597_amd import EtdmError
    wl = make_config(1)
    h, _ = make_handle(wl, "fp64")
    A = torch.zeros(h.n_param, dtype=torch.float64, device="cuda:0")
    rho = torch.empty(64 * 64, dtype=torch.float64, device="cuda:0")
    with pytest.raises(EtdmError):
        h.density(A, rho)
    h.close()
