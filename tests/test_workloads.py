"""Properties of the seeded synthetic inputs (shapes, symmetry, determinism)."""
import numpy as np
import pytest

from workloads import make_config, tiny_complex, tiny_real
from workloads.gen import config2_sizes


def test_config1_recipe():
    wl = make_config(1)
    (inst,) = wl.instances
    assert (inst.M, inst.N) == (64, 16)
    assert np.allclose(np.diag(inst.H0), np.linspace(-2, 2, 64))
    assert np.array_equal(inst.H0, inst.H0.T)
    assert np.abs(inst.C0.T @ inst.C0 - np.eye(64)).max() < 1e-13
    assert inst.A.shape == (16, 48) and 0.04 < inst.A.std() < 0.06
    assert np.array_equal(inst.f, np.r_[np.full(16, 2.0), np.zeros(48)])


def test_deterministic():
    a, b = make_config(1), make_config(1)
    assert np.array_equal(a.instances[0].C0, b.instances[0].C0)
    assert np.array_equal(a.instances[0].A, b.instances[0].A)


def test_config2_sizes():
    s = config2_sizes()
    assert s.size == 148 and s.min() >= 20 and s.max() <= 400
    wl = make_config(2, n_inst=5)
    for inst, M in zip(wl.instances, s[:5]):
        assert inst.M == M and inst.N == round(M / 5)


def test_config3_block_sparse():
    wl = make_config(3)
    (inst,) = wl.instances
    assert (inst.M, inst.N) == (1472, 256)
    b = inst.H0_bsr
    H = b.to_dense()
    assert np.array_equal(H, H.T)
    frac = b.col_idx.size / 64 ** 2
    assert 0.3 < frac < 0.7  # roughly half of the blocks within 6 A in a 12.4 A box
    assert np.all(np.diff(b.row_ptr) >= 1)


def test_config4_crystal():
    wl = make_config(4, nk=4)
    assert wl.kind == "complex_full" and wl.couple
    full = make_config(4)
    assert len(full.instances) == 64
    ne = sum(i.weight * i.f.sum() for i in full.instances)
    assert abs(ne - 40.0) < 1e-9
    for inst in wl.instances:
        assert np.abs(inst.H0 - inst.H0.conj().T).max() < 1e-14
        assert np.abs(inst.A + inst.A.conj().T).max() < 1e-15
        assert np.abs(inst.C0.conj().T @ inst.C0 - np.eye(208)).max() < 1e-13
        assert np.all((inst.f >= 0) & (inst.f <= 2))
    fr = np.concatenate([i.f for i in full.instances])
    assert np.any((fr > 1e-6) & (fr < 2 - 1e-6))  # some fractional occupations


def test_tiny_generators():
    wl = tiny_real(10, 3, n_inst=2)
    assert len(wl.instances) == 2
    wc = tiny_complex(6, nk_side=1)
    assert wc.instances[0].H0.shape == (6, 6)
