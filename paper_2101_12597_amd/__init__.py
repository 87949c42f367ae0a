"""MI355X (gfx950) implementation of the ETDM energy+gradient hot path.

The computation lives in the HIP library ``libetdm.so`` (C ABI in
``include/etdm.h``); this package holds its sources (``csrc/``), the build
script and a thin ctypes binding.
"""
from .etdm import (  # noqa: F401
    COMPLEX_FULL,
    EXPORTS,
    LIB_PATH,
    PRECISIONS,
    REAL_OV,
    EtdmError,
    Handle,
    LbfgsParams,
    energy_grad_static,
    etdm_energy,
    lbfgs_defaults,
    load_library,
)
