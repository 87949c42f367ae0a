"""CPU-side checks of the C ABI: the library builds/loads and exports every
symbol that include/etdm.h declares; host-side argument validation (no GPU
compute is launched)."""
import ctypes
import os
import re

import pytest


def declared_symbols(root):
    text = open(os.path.join(root, "include", "etdm.h")).read()
    # function declarations: a return type at the start of a line, then the name
    pat = r"^(?:const\s+)?(?:void|int64_t|size_t|char|etdm_status)\s*\*?\s*(etdm_[a-z_]+)\s*\("
    return sorted(set(re.findall(pat, text, flags=re.M)))


def test_header_declares_expected_entry_points(repo_root):
    syms = declared_symbols(repo_root)
    for s in ["etdm_create", "etdm_destroy", "etdm_expm", "etdm_energy_grad", "etdm_lbfgs_step",
              "etdm_set_reference", "etdm_sync_status", "etdm_status_string", "etdm_last_error",
              "etdm_lbfgs_state_bytes", "etdm_lbfgs_get_state", "etdm_lbfgs_set_state"]:
        assert s in syms


def test_library_exports_every_declared_symbol(repo_root):
    from paper_2101_12597_amd import LIB_PATH, load_library
    if not os.path.exists(LIB_PATH):
        pytest.skip("libetdm.so not built (run __graft_entry__.build())")
    lib = load_library()
    for s in declared_symbols(repo_root):
        assert hasattr(lib, s), s


def test_host_only_calls(repo_root):
    from paper_2101_12597_amd import LIB_PATH, load_library, lbfgs_defaults
    if not os.path.exists(LIB_PATH):
        pytest.skip("libetdm.so not built")
    lib = load_library()
    assert lib.etdm_status_string(0) == b"ok"
    assert lib.etdm_status_string(-5) == b"eigensolver did not converge"
    p = lbfgs_defaults()
    assert (p.m, p.c1, p.c2, p.delta, p.sigma, p.eps, p.gamma, p.reset_every) == \
        (3, 1e-4, 0.9, 0.1, 0.9, 1e-6, 0.25, 20)
    # null handle and null descriptor are rejected before any device work
    assert lib.etdm_create(None, None, None, None, None, None) == -1
    assert lib.etdm_energy_grad(None, None, None, None, None) == -1
    assert lib.etdm_destroy(None) == -1
    assert lib.etdm_param_count(None) == 0
    assert lib.etdm_lbfgs_state_bytes(None) == 0
    assert lib.etdm_lbfgs_get_state(None, None, None) == -1
    assert lib.etdm_lbfgs_set_state(None, None, None) == -1


@pytest.mark.parametrize("field,bad", [("gemm_tuning", -1), ("gemm_tuning", 7), ("gradient", -1),
                                       ("gradient", 2), ("expm_method", -1), ("expm_method", 2),
                                       ("expm_method", 1), ("odd_lambda", 0.5), ("odd_lambda", float("nan"))])
def test_create_rejects_bad_mode_fields(repo_root, field, bad):
    """gemm_tuning outside 0..6, gradient or expm_method outside {0, 1}, and scaling and
    squaring or the orbital-dependent term on the real kind (both need COMPLEX_FULL),
    and a non-finite term strength are argument errors, found before any device call."""
    from paper_2101_12597_amd import LIB_PATH, load_library
    from paper_2101_12597_amd.etdm import _Desc
    if not os.path.exists(LIB_PATH):
        pytest.skip("libetdm.so not built")
    lib = load_library()
    M = (ctypes.c_int32 * 1)(64)
    N = (ctypes.c_int32 * 1)(16)
    f = (ctypes.c_double * 64)(*([2.0] * 16 + [0.0] * 48))
    d = _Desc()
    d.n_inst = 1
    d.M = M
    d.N = N
    d.kind = 0
    d.precision = 4
    setattr(d, field, bad)
    h = ctypes.c_void_p()
    dummy = ctypes.c_void_p(8)  # never dereferenced: validation fails first
    assert lib.etdm_create(ctypes.byref(h), ctypes.byref(d), dummy, dummy, f, None) == -1
    assert h.value is None


def test_create_rejects_scaling_and_squaring_beyond_its_size(repo_root):
    """Scaling and squaring serves complex instances up to M = 1024 (the column tiles of
    its norm and the panels of its solve are sized for that); a larger one is a shape
    error, found before any device call."""
    from paper_2101_12597_amd import LIB_PATH, load_library
    from paper_2101_12597_amd.etdm import _Desc
    if not os.path.exists(LIB_PATH):
        pytest.skip("libetdm.so not built")
    lib = load_library()
    m = 1025
    M = (ctypes.c_int32 * 1)(m)
    N = (ctypes.c_int32 * 1)(m)
    f = (ctypes.c_double * m)(*([2.0] * 8 + [0.0] * (m - 8)))
    d = _Desc()
    d.n_inst = 1
    d.M = M
    d.N = N
    d.kind = 1  # ETDM_COMPLEX_FULL
    d.precision = 0  # ETDM_FP64
    d.expm_method = 1
    h = ctypes.c_void_p()
    dummy = ctypes.c_void_p(8)  # never dereferenced: validation fails first
    assert lib.etdm_create(ctypes.byref(h), ctypes.byref(d), dummy, dummy, f, None) == -2  # ETDM_E_SHAPE
    assert h.value is None
