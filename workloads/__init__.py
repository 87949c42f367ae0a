"""Seeded synthetic inputs for the ETDM energy+gradient path.

This package only draws random numbers and lays them out (Hamiltonians,
reference orbitals, occupations, rotation parameters).  It holds none of the
method's arithmetic, so both the CPU oracle and the GPU path can consume the
same bytes without sharing any computation.
"""
from .gen import (  # noqa: F401
    Instance,
    Workload,
    make_config,
    tiny_real,
    tiny_complex,
    with_overlap,
    CONFIG_NAMES,
)
