"""Seeded synthetic inputs shared, as data, by the oracle and the HIP path.

This module draws random numbers and arranges them into arrays; it holds none
of the method's arithmetic (no Dirac operator, no smearing, no solver, no
contraction).  Both the CPU oracle and the GPU library receive the arrays made
here and nothing else from it.

Array conventions (the library's boundary layout):
  site index  s = x + Lx*(y + Ly*(z + Lz*t))      (mu = 0,1,2,3 are x,y,z,t)
  links       U[s][mu][row][col]                   complex128
  spinors     psi[s][spin][colour]                 complex128
  cut masks   cut_after[mu][x] in {0,1}: 1 means the face between x and
              x+1 (mod L_mu) in direction mu is a domain boundary.

The paper's ensemble (Nf=3+1 Wilson-clover, 96x32^3, open time boundaries;
Results section) is not available; the presets below are synthetic stand-ins
whose shapes follow the method's distillation set-up at reduced size.
"""
from __future__ import annotations

import dataclasses
import numpy as np

__all__ = [
    "Preset", "PRESETS", "gell_mann", "gauge_field", "random_su3",
    "random_spinor", "tiling_cuts", "offset_tiling_cuts", "volume",
]


def volume(dims):
    return int(np.prod(dims))


def gell_mann() -> np.ndarray:
    """The eight Gell-Mann matrices lambda_a (shape [8,3,3])."""
    l = np.zeros((8, 3, 3), dtype=np.complex128)
    l[0][0, 1] = l[0][1, 0] = 1
    l[1][0, 1] = -1j
    l[1][1, 0] = 1j
    l[2][0, 0] = 1
    l[2][1, 1] = -1
    l[3][0, 2] = l[3][2, 0] = 1
    l[4][0, 2] = -1j
    l[4][2, 0] = 1j
    l[5][1, 2] = l[5][2, 1] = 1
    l[6][1, 2] = -1j
    l[6][2, 1] = 1j
    l[7][0, 0] = l[7][1, 1] = 1 / np.sqrt(3)
    l[7][2, 2] = -2 / np.sqrt(3)
    return l


def _reunitarise(m: np.ndarray) -> np.ndarray:
    """Gram-Schmidt on rows 0,1; row 2 = conj(row0 x row1): exact SU(3)."""
    r0 = m[..., 0, :]
    r0 = r0 / np.linalg.norm(r0, axis=-1, keepdims=True)
    r1 = m[..., 1, :]
    r1 = r1 - np.sum(np.conj(r0) * r1, axis=-1, keepdims=True) * r0
    r1 = r1 / np.linalg.norm(r1, axis=-1, keepdims=True)
    r2 = np.conj(np.cross(r0, r1))
    return np.stack([r0, r1, r2], axis=-2)


def _expi_hermitian(h: np.ndarray) -> np.ndarray:
    """exp(i h) for a batch of hermitian 3x3 matrices via eigh."""
    w, v = np.linalg.eigh(h)
    return np.einsum("...ij,...j,...kj->...ik", v, np.exp(1j * w), np.conj(v))


def gauge_field(dims, eps: float, seed: int, chunk: int = 1 << 18) -> np.ndarray:
    """U_mu(x) = exp(i eps sum_a r_a T_a), T_a = lambda_a/2, r_a ~ N(0,1) iid,
    then reunitarised.  Returns complex128 [V][4][3][3]."""
    V = volume(dims)
    rng = np.random.Generator(np.random.PCG64(seed))
    T = gell_mann() / 2
    n = V * 4
    out = np.empty((n, 3, 3), dtype=np.complex128)
    for a in range(0, n, chunk):
        b = min(n, a + chunk)
        r = rng.standard_normal((b - a, 8))
        h = eps * np.einsum("na,aij->nij", r, T)
        out[a:b] = _reunitarise(_expi_hermitian(h))
    return out.reshape(V, 4, 3, 3)


def random_su3(n: int, seed: int) -> np.ndarray:
    """n Haar-ish random SU(3) matrices (QR of a complex Gaussian, then
    phase-fixed to det 1).  Used for gauge transformations in tests."""
    rng = np.random.Generator(np.random.PCG64(seed))
    z = rng.standard_normal((n, 3, 3)) + 1j * rng.standard_normal((n, 3, 3))
    q, r = np.linalg.qr(z)
    d = np.diagonal(r, axis1=-2, axis2=-1)
    q = q * (d / np.abs(d))[:, None, :]
    det = np.linalg.det(q)
    q = q / (det ** (1.0 / 3.0))[:, None, None]
    return _reunitarise(q)


def random_spinor(V: int, n: int, seed: int) -> np.ndarray:
    """n Gaussian spinor fields, N(0,1) per real component: complex128 [n][V][4][3]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    re = rng.standard_normal((n, V, 4, 3))
    im = rng.standard_normal((n, V, 4, 3))
    return re + 1j * im


def random_colour_vectors(T: int, nv: int, Vs: int, seed: int) -> np.ndarray:
    """Seeded stand-ins for smearing vectors: nv complex Gaussian colour fields
    per timeslice, each of unit norm, complex128 [T][nv][Vs][3] (the layout of
    the eigenvectors).  V^+ D^-1 V is defined for any V, so solver and
    projection checks can use these in place of Laplacian eigenvectors."""
    rng = np.random.Generator(np.random.PCG64(seed))
    v = rng.standard_normal((T, nv, Vs, 3)) + 1j * rng.standard_normal((T, nv, Vs, 3))
    return v / np.sqrt((np.abs(v) ** 2).sum(axis=(2, 3), keepdims=True))


def random_spinor_device(V: int, n: int, seed: int, device="cuda:0"):
    """n Gaussian spinor fields, N(0,1) per real component, drawn on the GPU by
    torch's seeded generator (for multi-gigabyte blocks that need not pass
    through host memory): complex128 torch tensor [n][V][4][3]."""
    import torch
    g = torch.Generator(device=device).manual_seed(int(seed))
    re = torch.randn((n, V, 4, 3), generator=g, device=device, dtype=torch.float64)
    im = torch.randn((n, V, 4, 3), generator=g, device=device, dtype=torch.float64)
    return torch.complex(re, im)


def tiling_cuts(dims, block) -> np.ndarray:
    """Cut masks for a regular tiling with block extent block[mu] along mu
    (block[mu] == dims[mu] means no cut in that direction).  Returns uint8
    [4][max(dims)], row mu valid for x < dims[mu]."""
    Lmax = max(dims)
    cut = np.zeros((4, Lmax), dtype=np.uint8)
    for mu in range(4):
        L, b = dims[mu], block[mu]
        if b >= L:
            continue
        for x in range(L):
            if (x + 1) % b == 0:
                cut[mu, x] = 1
    return cut


def offset_tiling_cuts(dims, block) -> np.ndarray:
    """Tiling offset by half a block with the wrap face cut, giving uneven
    domains (e.g. 24 with block 6: extents 3,6,6,6,3)."""
    Lmax = max(dims)
    cut = np.zeros((4, Lmax), dtype=np.uint8)
    for mu in range(4):
        L, b = dims[mu], block[mu]
        if b >= L:
            continue
        h = b // 2
        for x in range(L):
            if (x + 1 - h) % b == 0:
                cut[mu, x] = 1
        cut[mu, L - 1] = 1
    return cut


@dataclasses.dataclass(frozen=True)
class Preset:
    name: str
    dims: tuple          # (Lx, Ly, Lz, Lt)
    eps: float           # link spread
    ape_steps: int
    ape_alpha: float
    kappa: float
    csw: float
    nv: int
    block: tuple         # domain extents
    seed: int
    bc: tuple = (1, 1, 1, -1)   # periodic space, antiperiodic time


PRESETS = {
    # Plain FP64 chain, small enough for the oracle to run everything.
    "plain_4x4x4x4": Preset("plain_4x4x4x4", (4, 4, 4, 4), 0.3, 0, 0.5, 0.120, 1.0, 4,
                            (2, 2, 2, 2), 1),
    # Mixed-precision production shape.
    "prec_16x16x16x32": Preset("prec_16x16x16x32", (16, 16, 16, 32), 0.25, 5, 0.5, 0.125, 1.5,
                               32, (4, 4, 4, 8), 2),
    # Large multi-RHS shape.
    "batch_24x24x24x48": Preset("batch_24x24x24x48", (24, 24, 24, 48), 0.25, 5, 0.5, 0.126, 1.6,
                                64, (6, 6, 8, 12), 3),
    # Production-sized lattice.
    "prod_32x32x32x64": Preset("prod_32x32x32x64", (32, 32, 32, 64), 0.2, 10, 0.5, 0.127, 1.7,
                               128, (8, 8, 8, 16), 500),
}
