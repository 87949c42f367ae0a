"""Pack a workload into the flat host arrays of the library's C ABI layout
(instances back to back, row-major, complex as interleaved float64 pairs)."""
from __future__ import annotations

from typing import Dict, List

import numpy as np


def _flat(x: np.ndarray) -> np.ndarray:
    x = np.ascontiguousarray(x)
    return x.view(np.float64).ravel() if np.iscomplexobj(x) else x.ravel()


def pack(wl, use_bsr: bool = False) -> Dict[str, object]:
    out: Dict[str, object] = {}
    out["kind"] = wl.kind
    out["M"] = [inst.M for inst in wl.instances]
    out["N"] = [inst.N for inst in wl.instances]
    out["weights"] = [inst.weight for inst in wl.instances]
    out["f"] = np.concatenate([inst.f for inst in wl.instances])
    out["C0"] = np.concatenate([_flat(inst.C0) for inst in wl.instances])
    if use_bsr:
        blocks, rps, cis = [], [], []
        bs = wl.instances[0].H0_bsr.block
        for inst in wl.instances:
            b = inst.H0_bsr
            assert b.block == bs
            blocks.append(b.blocks.ravel())
            rps.append(b.row_ptr)
            cis.append(b.col_idx)
        out["H0"] = np.concatenate(blocks)
        out["bsr"] = (bs, np.concatenate(rps), np.concatenate(cis))
    else:
        out["H0"] = np.concatenate([_flat(inst.h0_dense()) for inst in wl.instances])
        out["bsr"] = None
    out["A"] = pack_params(wl, [inst.A if wl.kind == "real_ov" else np.triu(inst.A)
                                for inst in wl.instances])
    out["S"] = (np.concatenate([_flat(inst.S) for inst in wl.instances])
                if any(inst.S is not None for inst in wl.instances) else None)
    return out


def pack_params(wl, params: List[np.ndarray]) -> np.ndarray:
    return np.concatenate([_flat(p) for p in params]) if params else np.zeros(0)


def unpack_params(wl, vec: np.ndarray) -> List[np.ndarray]:
    out, o = [], 0
    for inst in wl.instances:
        if wl.kind == "real_ov":
            n = inst.N * (inst.M - inst.N)
            out.append(vec[o:o + n].reshape(inst.N, inst.M - inst.N).copy())
        else:
            n = 2 * inst.M * inst.M
            out.append(vec[o:o + n].view(np.complex128).reshape(inst.M, inst.M).copy())
        o += n
    return out


def unpack_square(wl, vec: np.ndarray) -> List[np.ndarray]:
    """Split a packed array of M x M matrices (real or complex) per instance."""
    out, o = [], 0
    for inst in wl.instances:
        if wl.kind == "real_ov":
            n = inst.M * inst.M
            out.append(vec[o:o + n].reshape(inst.M, inst.M).copy())
        else:
            n = 2 * inst.M * inst.M
            out.append(vec[o:o + n].view(np.complex128).reshape(inst.M, inst.M).copy())
        o += n
    return out
