"""Seeded generators for the five synthetic ETDM workloads and small test cases.

Every array is FP64 (or complex128) on the host.  Seeds come from
``numpy.random.SeedSequence([12597, cfg, inst, stream])`` with the streams

    0  Hamiltonian entries        1  reference orbitals C0
    2  rotation parameters (A)    3  molecule positions
    4  periodic hopping blocks    9  instance sizes (ragged batch)

Workload recipes (stand-ins for the paper's G2 molecules, ionic crystals and
liquid-water snapshots, which are not available here):

* model Hamiltonian "chain": H0 = diag(linspace(-2, 2, M)) plus a symmetric
  off-diagonal part with entries N(0, 0.1^2) * exp(-|mu - nu| / 8), drawn on the
  strict upper triangle and mirrored;
* "water box": M = 23 * n_mol basis functions, 23 x 23 diagonal blocks with
  upper-triangle entries N(0, 0.5^2) mirrored, off-diagonal blocks
  N(0, 0.05^2) * exp(-d / 2 A) for minimum-image centre distances d < 6 A,
  H_JI = H_IJ^T; N = 4 occupied orbitals per molecule;
* "crystal": complex Hermitian H0(k) = H_on + sum_R T_R exp(i 2 pi n.R / 4)
  over the 26 neighbour cells R in {-1,0,1}^3 minus 0 of a 4x4x4 Gamma-centred
  grid, T_R ~ N(0, 0.1^2) exp(-|R|), T_-R = T_R^T, fractional Fermi-Dirac
  occupations (kT = 0.01 Ha, 40 electrons per cell, spin factor 2).

Reference orbitals are Haar-distributed (QR of a Gaussian matrix with the
signs/phases of diag(R) moved into Q).  Occupied columns come first.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

BASE_SEED = 12597
HUBBARD_U = 0.5
F_OCC = 2.0

CONFIG_NAMES = {
    1: "chain M=64 N=16 real (single molecule)",
    2: "148 ragged molecules M~U[20,400] N=round(M/5) real",
    3: "64-water box M=1472 N=256 real, block-sparse H0",
    4: "crystal 4x4x4 k-grid M=208 complex, Fermi-Dirac f",
    5: "576-water box M=13248 N=2304 real, block-sparse H0",
}


def rng_for(cfg: int, inst: int, stream: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([BASE_SEED, cfg, inst, stream]))


@dataclass
class BSR:
    """Block-sparse row storage of a symmetric matrix with square blocks."""

    block: int
    row_ptr: np.ndarray  # int32 [n_block_rows + 1]
    col_idx: np.ndarray  # int32 [nnzb]
    blocks: np.ndarray  # float64 [nnzb, block, block] (row-major blocks)

    @property
    def n(self) -> int:
        return (len(self.row_ptr) - 1) * self.block

    def to_dense(self) -> np.ndarray:
        b = self.block
        out = np.zeros((self.n, self.n))
        for I in range(len(self.row_ptr) - 1):
            for p in range(self.row_ptr[I], self.row_ptr[I + 1]):
                J = self.col_idx[p]
                out[I * b:(I + 1) * b, J * b:(J + 1) * b] = self.blocks[p]
        return out


@dataclass
class Instance:
    M: int
    N: int  # number of columns with f > 0 (occupied columns come first)
    f: np.ndarray  # [M]
    C0: np.ndarray  # [M, M] real or complex, orthonormal columns
    A: np.ndarray  # real ov block B [N, M-N]  or complex skew-Hermitian [M, M]
    weight: float = 1.0
    H0: Optional[np.ndarray] = None  # dense [M, M]
    H0_bsr: Optional[BSR] = None
    S: Optional[np.ndarray] = None  # overlap of a non-orthogonal basis [M, M] (None: S = I)

    def h0_dense(self) -> np.ndarray:
        if self.H0 is not None:
            return self.H0
        return self.H0_bsr.to_dense()


@dataclass
class Workload:
    cfg: int
    name: str
    kind: str  # "real_ov" or "complex_full"
    hubbard_U: float
    couple: bool  # Hubbard term on the weight-averaged diagonal of all instances
    instances: List[Instance] = field(default_factory=list)

    @property
    def n_electrons(self) -> float:
        return float(sum(inst.weight * inst.f.sum() for inst in self.instances))


# --------------------------------------------------------------------------
# building blocks (random draws and layout only)
# --------------------------------------------------------------------------

def haar_orthogonal(M: int, rng: np.random.Generator) -> np.ndarray:
    G = rng.standard_normal((M, M))
    Q, R = np.linalg.qr(G)
    d = np.sign(np.diag(R))
    d[d == 0] = 1.0
    return Q * d[None, :]


def haar_unitary(M: int, rng: np.random.Generator) -> np.ndarray:
    G = (rng.standard_normal((M, M)) + 1j * rng.standard_normal((M, M))) / np.sqrt(2.0)
    Q, R = np.linalg.qr(G)
    d = np.diag(R)
    ph = d / np.where(np.abs(d) == 0, 1.0, np.abs(d))
    return Q * ph[None, :]


def chain_hamiltonian(M: int, rng: np.random.Generator) -> np.ndarray:
    H = np.diag(np.linspace(-2.0, 2.0, M))
    iu, ju = np.triu_indices(M, 1)
    vals = rng.normal(0.0, 0.1, size=iu.size) * np.exp(-np.abs(iu - ju) / 8.0)
    H[iu, ju] = vals
    H[ju, iu] = vals
    return H


def water_box_hamiltonian(cfg: int, n_mol: int, box: float, bs: int = 23,
                          cutoff: float = 6.0) -> BSR:
    pos = rng_for(cfg, 0, 3).uniform(0.0, box, size=(n_mol, 3))
    rng = rng_for(cfg, 0, 0)
    dblk = rng.normal(0.0, 0.5, size=(n_mol, bs, bs))
    dblk = np.triu(dblk) + np.transpose(np.triu(dblk, 1), (0, 2, 1))
    I, J = np.triu_indices(n_mol, 1)
    dv = pos[J] - pos[I]
    dv -= box * np.round(dv / box)
    dist = np.sqrt((dv * dv).sum(axis=1))
    keep = dist < cutoff
    I, J, dist = I[keep], J[keep], dist[keep]
    oblk = rng.normal(0.0, 0.05, size=(I.size, bs, bs)) * np.exp(-dist / 2.0)[:, None, None]
    rows: List[List[Tuple[int, np.ndarray]]] = [[(r, dblk[r])] for r in range(n_mol)]
    for p in range(I.size):
        rows[I[p]].append((int(J[p]), oblk[p]))
        rows[J[p]].append((int(I[p]), oblk[p].T))
    row_ptr = [0]
    col_idx: List[int] = []
    blocks: List[np.ndarray] = []
    for r in range(n_mol):
        rows[r].sort(key=lambda t: t[0])
        for c, b in rows[r]:
            col_idx.append(c)
            blocks.append(b)
        row_ptr.append(len(col_idx))
    return BSR(bs, np.asarray(row_ptr, np.int32), np.asarray(col_idx, np.int32),
               np.ascontiguousarray(np.stack(blocks)))


def binary_occupations(M: int, N: int) -> np.ndarray:
    f = np.zeros(M)
    f[:N] = F_OCC
    return f


def ov_parameters(N: int, Nv: int, rng: np.random.Generator, scale: float = 0.05) -> np.ndarray:
    return rng.normal(0.0, scale, size=(N, Nv))


def skew_hermitian(M: int, rng: np.random.Generator, scale: float = 0.05) -> np.ndarray:
    re = rng.normal(0.0, scale, size=(M, M))
    im = rng.normal(0.0, scale, size=(M, M))
    d = rng.normal(0.0, scale, size=M)
    up = np.triu(re + 1j * im, 1)
    return up - up.conj().T + np.diag(1j * d)


def fermi_dirac_occupations(eps: np.ndarray, weights: np.ndarray, n_el: float,
                            kT: float) -> np.ndarray:
    """f = 2 / (1 + exp((eps - mu)/kT)), mu by bisection so that sum_k w_k sum_i f = n_el.

    Evaluated as 1 - tanh((eps - mu) / 2kT) to avoid overflow; values below 1e-15
    are set to 0 so every consumer sees the same occupations.
    """
    def occ(mu):
        return 1.0 - np.tanh((eps - mu) / (2.0 * kT))

    lo, hi = eps.min() - 1.0, eps.max() + 1.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if (weights[:, None] * occ(mid)).sum() > n_el:
            hi = mid
        else:
            lo = mid
    f = occ(0.5 * (lo + hi))
    f[f < 1e-15] = 0.0
    return f


# --------------------------------------------------------------------------
# the five workloads
# --------------------------------------------------------------------------

def _real_instance(cfg: int, inst: int, M: int, N: int, H0=None, H0_bsr=None) -> Instance:
    if H0 is None and H0_bsr is None:
        H0 = chain_hamiltonian(M, rng_for(cfg, inst, 0))
    C0 = haar_orthogonal(M, rng_for(cfg, inst, 1))
    B = ov_parameters(N, M - N, rng_for(cfg, inst, 2))
    return Instance(M=M, N=N, f=binary_occupations(M, N), C0=C0, A=B, H0=H0, H0_bsr=H0_bsr)


def config2_sizes(n_inst: int = 148) -> np.ndarray:
    return rng_for(2, 0, 9).integers(20, 401, size=n_inst)


def make_config(cfg: int, n_inst: Optional[int] = None, nk: Optional[int] = None) -> Workload:
    """Build workload ``cfg`` (1..5).  ``n_inst``/``nk`` truncate configs 2/4 for tests."""
    if cfg == 1:
        wl = Workload(1, CONFIG_NAMES[1], "real_ov", HUBBARD_U, False)
        wl.instances.append(_real_instance(1, 0, 64, 16))
        return wl
    if cfg == 2:
        sizes = config2_sizes(148)
        if n_inst is not None:
            sizes = sizes[:n_inst]
        wl = Workload(2, CONFIG_NAMES[2], "real_ov", HUBBARD_U, False)
        for i, M in enumerate(sizes):
            M = int(M)
            wl.instances.append(_real_instance(2, i, M, int(round(M / 5))))
        return wl
    if cfg in (3, 5):
        n_mol, box = (64, 12.4) if cfg == 3 else (576, 26.0)
        bsr = water_box_hamiltonian(cfg, n_mol, box)
        wl = Workload(cfg, CONFIG_NAMES[cfg], "real_ov", HUBBARD_U, False)
        wl.instances.append(_real_instance(cfg, 0, 23 * n_mol, 4 * n_mol, H0_bsr=bsr))
        return wl
    if cfg == 4:
        return crystal_workload(nk_side=4, M=208, n_el=40.0, nk_limit=nk)
    raise ValueError(f"unknown config {cfg}")


def crystal_hamiltonians(M: int, nk_side: int, cfg: int = 4) -> Tuple[np.ndarray, np.ndarray]:
    """H0(k) for a Gamma-centred nk_side^3 grid.  Returns (H [nk, M, M], weights [nk])."""
    H_on = chain_hamiltonian(M, rng_for(cfg, 0, 0))
    rng = rng_for(cfg, 0, 4)
    shells = [(a, b, c) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)
              if (a, b, c) > (0, 0, 0)]
    T = {}
    for R in shells:
        T[R] = rng.normal(0.0, 0.1, size=(M, M)) * np.exp(-np.sqrt(float(np.dot(R, R))))
    ks = [(a, b, c) for a in range(nk_side) for b in range(nk_side) for c in range(nk_side)]
    H = np.empty((len(ks), M, M), dtype=np.complex128)
    for ik, n in enumerate(ks):
        h = H_on.astype(np.complex128)
        for R, TR in T.items():
            ph = np.exp(2j * np.pi * np.dot(n, R) / nk_side)
            h = h + TR * ph + TR.T * np.conj(ph)
        H[ik] = h
    w = np.full(len(ks), 1.0 / len(ks))
    return H, w


def crystal_workload(nk_side: int = 4, M: int = 208, n_el: float = 40.0, kT: float = 0.01,
                     nk_limit: Optional[int] = None, cfg: int = 4) -> Workload:
    H, w = crystal_hamiltonians(M, nk_side, cfg)
    eps = np.stack([np.linalg.eigvalsh(h) for h in H])
    f_all = fermi_dirac_occupations(eps, w, n_el, kT)
    nk = H.shape[0] if nk_limit is None else min(nk_limit, H.shape[0])
    wl = Workload(cfg, CONFIG_NAMES.get(cfg, "crystal"), "complex_full", HUBBARD_U, True)
    for ik in range(nk):
        C0 = haar_unitary(M, rng_for(cfg, ik, 1))
        A = skew_hermitian(M, rng_for(cfg, ik, 2))
        f = f_all[ik]
        wl.instances.append(Instance(M=M, N=int((f > 0).sum()), f=f, C0=C0, A=A,
                                     weight=float(w[ik]), H0=H[ik]))
    return wl


# --------------------------------------------------------------------------
# small cases for tests
# --------------------------------------------------------------------------

def tiny_real(M: int, N: int, seed: int = 0, scale: float = 0.05, hubbard_U: float = HUBBARD_U,
              n_inst: int = 1) -> Workload:
    wl = Workload(100 + seed, f"tiny real M={M} N={N}", "real_ov", hubbard_U, False)
    for i in range(n_inst):
        H0 = chain_hamiltonian(M, rng_for(100 + seed, i, 0))
        C0 = haar_orthogonal(M, rng_for(100 + seed, i, 1))
        B = ov_parameters(N, M - N, rng_for(100 + seed, i, 2), scale)
        wl.instances.append(Instance(M=M, N=N, f=binary_occupations(M, N), C0=C0, A=B, H0=H0))
    return wl


def with_overlap(wl: Workload, strength: float = 0.15, seed: int = 0) -> Workload:
    """The same workload in a non-orthogonal basis: per instance an overlap
    S = I + strength * (symmetric / Hermitian with exponentially decaying entries),
    kept positive definite, and reference orbitals C0 = L^-H Q with S = L L^H (Cholesky)
    and Q the instance's orthonormal C0, so that C0^H S C0 = I.  H0 is reused as the
    Hamiltonian in the non-orthogonal basis."""
    for i, inst in enumerate(wl.instances):
        rng = rng_for(300 + seed, i, 0)
        M = inst.M
        R = rng.standard_normal((M, M))
        if wl.kind != "real_ov":
            R = R + 1j * rng.standard_normal((M, M))
        dist = np.abs(np.arange(M)[:, None] - np.arange(M)[None, :])
        R = R * np.exp(-dist / 3.0) / np.sqrt(M)
        S = np.eye(M) + strength * (R + R.conj().T) / 2.0
        lo = np.linalg.eigvalsh(S).min()
        if lo < 0.2:
            S = S + (0.2 - lo) * np.eye(M)
        L = np.linalg.cholesky(S)
        inst.S = S
        inst.C0 = np.linalg.solve(L.conj().T, inst.C0)
    wl.name += " (non-orthogonal basis)"
    return wl


def tiny_complex(M: int, nk_side: int = 2, n_el: Optional[float] = None, seed: int = 0,
                 kT: float = 0.01, hubbard_U: float = HUBBARD_U) -> Workload:
    if n_el is None:
        n_el = float(2 * max(1, M // 4))
    wl = crystal_workload(nk_side=nk_side, M=M, n_el=n_el, kT=kT, cfg=200 + seed)
    wl.hubbard_U = hubbard_U
    wl.name = f"tiny complex M={M} nk={nk_side ** 3}"
    return wl
