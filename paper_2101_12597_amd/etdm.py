"""Thin ctypes binding of ``libetdm.so`` (argument marshalling only).

Every step of the energy+gradient path runs in the HIP library; PyTorch is
used here only for device memory (tensors) and the current HIP stream.  The
library must have been built (``python -m paper_2101_12597_amd.build``); there
is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libetdm.so")

REAL_OV, COMPLEX_FULL = 0, 1
PRECISIONS = {"fp64": 0, "fp32": 1, "bf16x3": 2, "bf16x6": 3, "mixed": 4}

STATUS = {
    0: "ok", -1: "invalid argument", -2: "inconsistent shape", -3: "HIP runtime error",
    -4: "device allocation failed", -5: "eigensolver did not converge",
    -6: "non-finite energy or gradient", -7: "line search failed", -8: "invalid call sequence",
}


# the GEMM kernels of a real FP64 / BF16x6 stage, in the order of etdm_stage_kernel's times
GEMM_VARIANTS = ("tile64", "packed64", "packed128x64", "packed64x128", "packed128")


class EtdmError(RuntimeError):
    def __init__(self, code: int, detail: str = ""):
        self.code = code
        super().__init__(f"etdm error {code} ({STATUS.get(code, '?')}): {detail}")


class _Desc(ctypes.Structure):
    _fields_ = [
        ("n_inst", ctypes.c_int32),
        ("M", ctypes.POINTER(ctypes.c_int32)),
        ("N", ctypes.POINTER(ctypes.c_int32)),
        ("kind", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("hubbard_U", ctypes.c_double),
        ("couple", ctypes.c_int32),
        ("weights", ctypes.POINTER(ctypes.c_double)),
        ("h0_format", ctypes.c_int32),
        ("bsr_block", ctypes.c_int32),
        ("bsr_row_ptr", ctypes.POINTER(ctypes.c_int32)),
        ("bsr_col_idx", ctypes.POINTER(ctypes.c_int32)),
        ("gemm_tuning", ctypes.c_int32),
        ("gradient", ctypes.c_int32),
        ("expm_method", ctypes.c_int32),
        ("odd_lambda", ctypes.c_double),
        ("overlap", ctypes.c_void_p),
        ("want_rho", ctypes.c_int32),
    ]


class LbfgsParams(ctypes.Structure):
    _fields_ = [
        ("m", ctypes.c_int32),
        ("c1", ctypes.c_double), ("c2", ctypes.c_double), ("delta", ctypes.c_double),
        ("sigma", ctypes.c_double), ("eps", ctypes.c_double), ("gamma", ctypes.c_double),
        ("beta0", ctypes.c_double),
        ("reset_every", ctypes.c_int32),
        ("max_ls", ctypes.c_int32),
        ("reset_norm", ctypes.c_double),
    ]


class LbfgsInfo(ctypes.Structure):
    _fields_ = [
        ("iter", ctypes.c_int32), ("n_evals", ctypes.c_int32), ("alpha", ctypes.c_double),
        ("E", ctypes.c_double), ("gnorm", ctypes.c_double), ("flags", ctypes.c_int32),
    ]


EXPORTS = [
    "etdm_create", "etdm_destroy", "etdm_expm", "etdm_energy_grad", "etdm_set_reference",
    "etdm_lbfgs_defaults", "etdm_lbfgs_step", "etdm_sync_status", "etdm_status_string",
    "etdm_last_error", "etdm_param_count", "etdm_set_timing", "etdm_reset_timing",
    "etdm_stage_count", "etdm_stage_info", "etdm_stage_kernel", "etdm_set_graph", "etdm_density",
    "etdm_energy_grad_static",
]

_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libetdm.so and declare the C signatures (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2101_12597_amd.build`")
    L = ctypes.CDLL(path)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    L.etdm_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(_Desc), vp, vp,
                              ctypes.POINTER(dbl), vp]
    L.etdm_create.restype = i32
    L.etdm_destroy.argtypes = [vp]
    L.etdm_destroy.restype = i32
    L.etdm_expm.argtypes = [vp, vp, vp, vp]
    L.etdm_expm.restype = i32
    L.etdm_energy_grad.argtypes = [vp, vp, vp, vp, vp]
    L.etdm_energy_grad.restype = i32
    L.etdm_energy_grad_static.argtypes = [i32, i32, dbl, dbl, vp, vp, vp, vp, vp, vp, vp]
    L.etdm_energy_grad_static.restype = i32
    L.etdm_density.argtypes = [vp, vp, vp, vp]
    L.etdm_density.restype = i32
    L.etdm_set_reference.argtypes = [vp, vp, vp]
    L.etdm_set_reference.restype = i32
    L.etdm_lbfgs_defaults.argtypes = [ctypes.POINTER(LbfgsParams)]
    L.etdm_lbfgs_defaults.restype = None
    L.etdm_lbfgs_step.argtypes = [vp, ctypes.POINTER(LbfgsParams), vp, vp, vp,
                                  ctypes.POINTER(LbfgsInfo), vp]
    L.etdm_lbfgs_step.restype = i32
    L.etdm_lbfgs_state_bytes.argtypes = [vp]
    L.etdm_lbfgs_state_bytes.restype = ctypes.c_size_t
    L.etdm_lbfgs_get_state.argtypes = [vp, vp, vp]
    L.etdm_lbfgs_get_state.restype = i32
    L.etdm_lbfgs_set_state.argtypes = [vp, vp, vp]
    L.etdm_lbfgs_set_state.restype = i32
    L.etdm_sync_status.argtypes = [vp, vp]
    L.etdm_sync_status.restype = i32
    L.etdm_status_string.argtypes = [i32]
    L.etdm_status_string.restype = ctypes.c_char_p
    L.etdm_last_error.argtypes = [vp]
    L.etdm_last_error.restype = ctypes.c_char_p
    L.etdm_param_count.argtypes = [vp]
    L.etdm_param_count.restype = i64
    L.etdm_set_graph.argtypes = [vp, i32]
    L.etdm_set_graph.restype = i32
    L.etdm_set_timing.argtypes = [vp, i64]
    L.etdm_set_timing.restype = i32
    L.etdm_reset_timing.argtypes = [vp]
    L.etdm_reset_timing.restype = i32
    L.etdm_stage_count.argtypes = [vp]
    L.etdm_stage_count.restype = i32
    L.etdm_stage_info.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_char_p), ctypes.POINTER(i64),
                                  ctypes.POINTER(dbl), ctypes.POINTER(dbl), ctypes.POINTER(dbl)]
    L.etdm_stage_info.restype = i32
    L.etdm_stage_kernel.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_char_p), ctypes.POINTER(dbl)]
    L.etdm_stage_kernel.restype = i32
    _lib = L
    return L


def lbfgs_defaults() -> LbfgsParams:
    p = LbfgsParams()
    load_library().etdm_lbfgs_defaults(ctypes.byref(p))
    return p


def energy_grad_static(M: int, N: int, f_occ: float, hubbard_U: float, H0, C0, B, E, G, status,
                       stream=None) -> None:
    """etdm_energy_grad_static: E and dE/dB of one real occupied-virtual instance (dense
    H0, FP64) with every intermediate in the library's static device array (no handle, no
    allocation).  H0, C0: M x M float64; B, G: N x (M - N) float64; E: 2 float64 (the
    energy and the total); status: 1 int32 (0, or 1 eigensolver / 2 non-finite bits)."""
    import torch
    L = load_library()
    for t, n, dt in ((H0, M * M, torch.float64), (C0, M * M, torch.float64), (B, N * (M - N), torch.float64),
                     (G, N * (M - N), torch.float64), (E, 2, torch.float64), (status, 1, torch.int32)):
        if t.dtype != dt or t.numel() != n:
            raise ValueError(f"expected {n} elements of {dt}, got {t.numel()} of {t.dtype}")
    st = L.etdm_energy_grad_static(int(M), int(N), float(f_occ), float(hubbard_U), _dptr(H0), _dptr(C0), _dptr(B),
                                   _dptr(E), _dptr(G), _dptr(status), _stream_ptr(stream))
    if st != 0:
        raise EtdmError(st, "etdm_energy_grad_static")


def _stream_ptr(stream) -> int:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


def _dptr(t) -> int:
    if t is None:
        return 0
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous device tensor")
    return int(t.data_ptr())


class Handle:
    """Owns one etdm_handle (device copies of C0, H0, f and all workspaces).

    Parameters
    ----------
    M, N : per-instance basis sizes and occupied counts (N ignored for complex)
    kind : "real_ov" or "complex_full"
    precision : "fp64" | "fp32" | "bf16x3" | "bf16x6" | "mixed"
    H0 : device tensor, packed dense matrices (float64 / complex128), or the
         packed BSR blocks when ``bsr`` = (block, row_ptr, col_idx) is given
    C0 : device tensor, packed M x M reference orbitals
    f : host array of occupations, packed [sum M]
    gemm_tuning : kernel choice of the FP64 / BF16x6 GEMM stages: 0 = time the five
                  kernels at creation and keep the fastest, 1 = fixed size rule,
                  2 = packed 128 x 128, 3 = grouped 64 x 64, 4 = packed 64 x 64,
                  5 = packed 128 x 64, 6 = packed 64 x 128
    gradient : "exact" (Eq. gradients) or "approx" (G ~ L^T, Eq. app_grad)
    expm : "eig" (eigendecomposition of iA, Eq. ed) or "ss" (scaling and squaring with a
           Pade approximant, Eq. ss, and its Frechet derivative for the exact gradient;
           complex kind)
    odd_lambda : strength of the orbital-dependent model term (complex kind; 0 = off)
    overlap : device tensor, the overlap S of a non-orthogonal basis (layout of a dense H0),
              or None for an orthonormal basis
    want_rho : also hold the workspace of density() (M x M per instance)
    """

    def __init__(self, M: Sequence[int], N: Optional[Sequence[int]], kind: str, precision: str,
                 hubbard_U: float, H0, C0, f: np.ndarray, couple: bool = False,
                 weights: Optional[Sequence[float]] = None, bsr=None, stream=None,
                 gemm_tuning: int = 0, gradient: str = "exact", expm: str = "eig",
                 odd_lambda: float = 0.0, overlap=None, want_rho: bool = False):
        L = load_library()
        self._L = L
        n = len(M)
        self.kind = REAL_OV if kind == "real_ov" else COMPLEX_FULL
        self.M = np.ascontiguousarray(M, dtype=np.int32)
        self.N = np.ascontiguousarray(N if N is not None else M, dtype=np.int32)
        self._w = np.ascontiguousarray(weights if weights is not None else np.ones(n), dtype=np.float64)
        self._f = np.ascontiguousarray(f, dtype=np.float64)
        d = _Desc()
        d.n_inst = n
        d.M = self.M.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        d.N = self.N.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        d.kind = self.kind
        d.precision = PRECISIONS[precision]
        d.hubbard_U = float(hubbard_U)
        d.couple = int(bool(couple))
        d.weights = self._w.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        d.gemm_tuning = int(gemm_tuning)
        if gradient not in ("exact", "approx"):
            raise ValueError("gradient must be 'exact' or 'approx'")
        d.gradient = 1 if gradient == "approx" else 0
        if expm not in ("eig", "ss"):
            raise ValueError("expm must be 'eig' or 'ss'")
        d.expm_method = 1 if expm == "ss" else 0
        d.odd_lambda = float(odd_lambda)
        d.overlap = _dptr(overlap) if overlap is not None else None
        d.want_rho = int(bool(want_rho))
        if bsr is not None:
            blk, rp, ci = bsr
            self._rp = np.ascontiguousarray(rp, dtype=np.int32)
            self._ci = np.ascontiguousarray(ci, dtype=np.int32)
            d.h0_format = 1
            d.bsr_block = int(blk)
            d.bsr_row_ptr = self._rp.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
            d.bsr_col_idx = self._ci.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        h = ctypes.c_void_p()
        st = L.etdm_create(ctypes.byref(h), ctypes.byref(d), _dptr(H0), _dptr(C0),
                           self._f.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _stream_ptr(stream))
        if st != 0:
            raise EtdmError(st, "etdm_create")
        self._h = h
        self.n_inst = n
        self.n_param = int(L.etdm_param_count(h))

    # -- helpers -------------------------------------------------------------
    def _check(self, st: int, what: str):
        if st != 0:
            detail = self._L.etdm_last_error(self._h)
            raise EtdmError(st, f"{what}: {detail.decode() if detail else ''}")

    def _check_param(self, A):
        if A.dtype.itemsize * A.numel() != 8 * self.n_param:
            raise ValueError(f"parameter tensor has {A.numel()} elements of {A.dtype}, "
                             f"expected {self.n_param} float64 units")

    # -- entry points --------------------------------------------------------
    def energy_grad(self, A, E, G, stream=None):
        self._check_param(A)
        self._check_param(G)
        if E.numel() != self.n_inst + 1 or E.dtype.itemsize != 8:
            raise ValueError("E must hold n_inst + 1 float64 values")
        self._check(self._L.etdm_energy_grad(self._h, _dptr(A), _dptr(E), _dptr(G),
                                             _stream_ptr(stream)), "etdm_energy_grad")

    def expm(self, A, U, stream=None):
        self._check_param(A)
        self._check(self._L.etdm_expm(self._h, _dptr(A), _dptr(U), _stream_ptr(stream)), "etdm_expm")

    def density(self, A, rho, stream=None):
        """rho = C F C^dagger of C = C0 exp(A), M x M per instance packed (float64 units:
        M^2 per real instance, 2 M^2 per complex one)."""
        self._check_param(A)
        n = sum((1 if self.kind == REAL_OV else 2) * int(m) * int(m) for m in self.M)
        if rho.dtype.itemsize * rho.numel() != 8 * n:
            raise ValueError(f"rho must hold {n} float64 units")
        self._check(self._L.etdm_density(self._h, _dptr(A), _dptr(rho), _stream_ptr(stream)), "etdm_density")

    def set_reference(self, A, stream=None):
        self._check_param(A)
        self._check(self._L.etdm_set_reference(self._h, _dptr(A), _stream_ptr(stream)),
                    "etdm_set_reference")

    def lbfgs_step(self, A, E, G, params: Optional[LbfgsParams] = None, stream=None) -> dict:
        self._check_param(A)
        self._check_param(G)
        info = LbfgsInfo()
        st = self._L.etdm_lbfgs_step(self._h, ctypes.byref(params) if params is not None else None,
                                     _dptr(A), _dptr(E), _dptr(G), ctypes.byref(info),
                                     _stream_ptr(stream))
        self._check(st, "etdm_lbfgs_step")
        return dict(iter=info.iter, n_evals=info.n_evals, alpha=info.alpha, E=info.E,
                    gnorm=info.gnorm, flags=info.flags)

    def lbfgs_state_bytes(self) -> int:
        """Size of the L-BFGS checkpoint image (0 before the first lbfgs_step)."""
        return int(self._L.etdm_lbfgs_state_bytes(self._h))

    def lbfgs_get_state(self, buf, stream=None):
        """Write the L-BFGS checkpoint into `buf`, a device uint8 tensor of
        lbfgs_state_bytes() bytes."""
        self._check_state_buffer(buf)
        self._check(self._L.etdm_lbfgs_get_state(self._h, _dptr(buf), _stream_ptr(stream)),
                    "etdm_lbfgs_get_state")

    def lbfgs_set_state(self, buf, stream=None):
        """Restore the L-BFGS run saved by lbfgs_get_state (same shapes and modes)."""
        self._check_state_buffer(buf)
        self._check(self._L.etdm_lbfgs_set_state(self._h, _dptr(buf), _stream_ptr(stream)),
                    "etdm_lbfgs_set_state")

    def _check_state_buffer(self, buf):
        import torch
        if not (isinstance(buf, torch.Tensor) and buf.is_cuda and buf.dtype == torch.uint8
                and buf.is_contiguous()):
            raise TypeError("the state buffer must be a contiguous uint8 tensor on the GPU")
        need = self.lbfgs_state_bytes()
        if need and buf.numel() < need:
            raise ValueError(f"state buffer holds {buf.numel()} bytes, {need} needed")

    def set_graph(self, enable: bool = True):
        """Replay the energy+gradient launch sequence from a captured HIP graph."""
        self._check(self._L.etdm_set_graph(self._h, int(bool(enable))), "etdm_set_graph")

    def set_timing(self, mask: int = -1):
        """Record HIP events around the selected stages (bit i = stage i)."""
        self._check(self._L.etdm_set_timing(self._h, int(mask)), "etdm_set_timing")

    def reset_timing(self):
        self._check(self._L.etdm_reset_timing(self._h), "etdm_reset_timing")

    def stage_info(self) -> list:
        """Per stage: name, timed launches, total ms, flops and bytes of one launch."""
        out = []
        for i in range(int(self._L.etdm_stage_count(self._h))):
            name = ctypes.c_char_p()
            n = ctypes.c_int64()
            ms, fl, by = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
            self._check(self._L.etdm_stage_info(self._h, i, ctypes.byref(name), ctypes.byref(n),
                                                ctypes.byref(ms), ctypes.byref(fl), ctypes.byref(by)),
                        "etdm_stage_info")
            out.append(dict(index=i, name=name.value.decode(), launches=n.value, total_ms=ms.value,
                            flops=fl.value, bytes=by.value))
        return out

    def stage_kernels(self) -> list:
        """Per stage: its GEMM kernel ("" if not a GEMM) and the launch times of the real
        FP64 / BF16x6 kernels measured by the tuning at creation (0 if not timed)."""
        out = []
        for i in range(int(self._L.etdm_stage_count(self._h))):
            v = ctypes.c_char_p()
            t = (ctypes.c_double * len(GEMM_VARIANTS))()
            self._check(self._L.etdm_stage_kernel(self._h, i, ctypes.byref(v), t), "etdm_stage_kernel")
            out.append(dict(index=i, kernel=v.value.decode(),
                            tuned_ms={name: t[k] for k, name in enumerate(GEMM_VARIANTS)}))
        return out

    def sync_status(self, stream=None):
        self._check(self._L.etdm_sync_status(self._h, _stream_ptr(stream)), "etdm_sync_status")

    def close(self):
        if getattr(self, "_h", None):
            self._L.etdm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _make_autograd():
    import torch

    class ETDMEnergy(torch.autograd.Function):
        """E(A) as a differentiable function of the packed parameters A.

        forward runs etdm_energy_grad once and keeps dE/dA; backward returns
        grad_output * dE/dA (the hand-written adjoint chain of the library).
        For complex parameters the returned gradient follows PyTorch's
        convention for real-valued functions of complex inputs,
        dE/dRe a + i dE/dIm a, which is exactly the library's G.
        """

        @staticmethod
        def forward(ctx, A, handle: Handle):
            A = A.contiguous()
            E = torch.empty(handle.n_inst + 1, dtype=torch.float64, device=A.device)
            G = torch.empty_like(A)
            handle.energy_grad(A, E, G)
            ctx.save_for_backward(G)
            return E[-1].clone()

        @staticmethod
        def backward(ctx, gE):
            (G,) = ctx.saved_tensors
            return gE * G, None

    return ETDMEnergy


_ETDMEnergy = None


def etdm_energy(A, handle: Handle):
    """Differentiable total energy E(A) (see ETDMEnergy)."""
    global _ETDMEnergy
    if _ETDMEnergy is None:
        _ETDMEnergy = _make_autograd()
    return _ETDMEnergy.apply(A, handle)
